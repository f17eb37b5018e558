// pond_kernels.hpp -- HIP kernels of the finite-volume PonD step (gfx950, wave64).
//
// Per step three launches on one stream:
//   dt_kernel    one thread per instance: dt = cfl / rate (rate from the previous update's
//                epilogue), clipped at t_end; advances the instance clock.
//   face_kernel  one thread per face (2D: per x-face and y-face owner position) with an
//                LDS-staged halo tile of phi-bar-plus cells; runs the predictor-corrector
//                iteration of the face frame (Sec. III.B.3) and writes the face state.
//   cell_kernel  one thread per cell: face populations converted into the cell frame, flux,
//                co-moving BGK update (Sec. III.B.2), FP64 conserved update, and the reframe
//                that opens the next step (Sec. III.B.4) with the CFL rate of the new frame.
//
// Cell state (SoA planes): FP64 conserved U = (rho, rho u, rho E), plus the non-equilibrium
// Grad coefficients of f~ (h2, h3) and g~ (h1, h2) in the cell's co-moving frame, in the
// precision R of the populations. g~'s h0 follows from the energy: the state carries exactly
// what the next step's reframe keeps.
// Face state (SoA planes, precision R): frame (u, T) -- also the next step's seed -- and
// all Hermite coefficients of phi at the face in that frame (f: degree 3, g: degree 2).
#pragma once

#include <stdint.h>

#include "pond_core.hpp"

namespace pond {

enum { BC_PERIODIC = 0, BC_OUTFLOW, BC_REFLECT, BC_FIXED, BC_FIXED_WINDOW, BC_SPLIT, BC_MOVING };

enum { ST_CELLS = 0, ST_CONV_CELLS, ST_FACES, ST_ITERS, ST_NONCONV, ST_FALLBACK, ST_DEPOUT, ST_ITMAX,
       ST_TAIL_FACES, ST_TAIL_ITERS, ST_N };

enum { ERR_NONPHYS = 1, ERR_DEPART = 2, ERR_NONCONV = 4 };

struct Params {
    int dim, nx, ny, n_inst;
    double x0, y0, dx, dy;
    double Cv, cfl, mu, tol;
    int limiter, max_iter;
    int bc[4];
    double bc_state[4][4], bc_alt[4][4], bc_param[4][4];
    double bc_speed[2]; // per axis: fastest particle speed of the prescribed boundary states
    int iter_split;     // 2D: iterations done in the face kernel before a face moves to the
                        // tail kernel (0: the face kernel runs every face to the end)
    int tail_cap;       // 2D: entries per sub-list of the tail list (one sub-list per axis
                        // and slot); tail_n = 2 * NSLOT * tail_cap entries in all
    int64_t tail_n;
    int vslots;         // copies of each instance's CFL-rate maximum (NSLOT for one
                        // instance, 1 for a batch, whose tubes spread the atomics anyway)
    int64_t ncell, nface, nfx;
};

template <typename R>
struct State {
    double *U;      // (D+2) x ncell
    R *H;           // non-equilibrium coefficients: 1D 4, 2D 12 planes x ncell
    R *F;           // face state: 1D 9, 2D 19 planes x nface
    int *fiter;     // per face: iterations | (nonconverged << 16) | (fallback << 17)
    const int *cell_inst;   // per cell (1D batch) or null
    const int *face_inst;   // per face (1D batch) or null
    const int64_t *cell_off; // per instance + 1
    const int64_t *pad_off;  // per instance: padded offset (cell_off + 4k)
    double *t, *tstart, *dt;   // per instance
    const double *dxk;         // per instance cell size (1D tubes), or null: P.dx
    unsigned long long *vmax;  // 2 x n_inst x vslots (step parity, instance, copy)
    unsigned long long *stats; // ST_N counters
    int *err;
    int *inst_err;             // per instance: nonzero once a step produced an invalid cell
    double *U2;                // semi-Lagrangian scheme: staging of the new state
    R *H2;
    // faces handed from the face kernel to the tail kernel (2D): face index, iteration
    // state (u_x, u_y, T, and the frame two iterations back: 6 planes of tail_n R), and
    // it | have_pp << 16 | restarted << 17. Entry (axis * NSLOT + slot) * tail_cap + pos:
    // every wave appends to the sub-list of its slot.
    int *tail_f;
    R *tail_s;
    int *tail_meta;
    int *tail_count;           // 2 x NSLOT sub-list lengths, cleared by dt_kernel
    int *seed_count;           // NSLOT lengths of the learned seed's face lists, cleared by
                               // dt_kernel (null without a network)
    int *tblock;               // per cell: nonzero while it is in the stencil of a face that
                               // the tail kernel finishes this step (0 between steps)
};

template <int D>
struct Layout;
template <>
struct Layout<1> {
    static constexpr int NH = 4;  // f h2 h3, g h1 h2
    static constexpr int NF = 9;  // u T | f h0..h3 | g h0..h2
    static constexpr int NL = 9;  // LDS: u s T rho fh2 fh3 g0 g1 g2
};
template <>
struct Layout<2> {
    static constexpr int NH = 12; // f h20 h11 h02 h30 h21 h12 h03, g h10 h01 h20 h11 h02
    static constexpr int NF = 19; // ux uy T | f 10 | g 6
    static constexpr int NL = 18; // LDS: ux uy s rho f(7) g(6) T
};

// ---------------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------------

PD unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Workgroups are dispatched to the 8 XCDs in turn by linear index (workgroup b runs on XCD
// b mod 8). xcd_tile(b, n) is a permutation of [0, n) that gives XCD x the x-th contiguous
// run of n/8 tiles (the first n mod 8 XCDs one more).
constexpr int NXCD = 8;
PD int xcd_tile(int b, int n)
{
    const int xcd = b % NXCD, local = b / NXCD;
    const int base = n / NXCD, rem = n % NXCD;
    return xcd < rem ? xcd * (base + 1) + local : rem * (base + 1) + (xcd - rem) * base + local;
}

// Counters and maxima are spread over NSLOT copies, one picked by the wave's global index:
// atomics on one address serialize in its L2 channel (about 10 ns each), so one counter
// hit once per wave would cost a kernel of 14,400 waves some 150 us. Readers combine the
// copies.
constexpr int NSLOT = 256;

PD unsigned wave_slot()
{
    const unsigned blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned nthr = blockDim.x * blockDim.y * blockDim.z;
    const unsigned tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    return (blk * ((nthr + 63) / 64) + tid / 64) & (NSLOT - 1);
}

PD bool wave_leader()
{
    return ((threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z)) & 63) == 0;
}

// all lanes of the wave must call these
PD void stat_add(unsigned long long *stats, int k, unsigned long long v)
{
    v = wave_sum(v);
    if (wave_leader() && v) atomicAdd(&stats[k * NSLOT + wave_slot()], v);
}

PD void stat_max(unsigned long long *stats, int k, unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    if (wave_leader() && v) atomicMax(&stats[k * NSLOT + wave_slot()], v);
}

// 32-bit forms, for counters whose wave total fits 32 bits
PD void stat_add32(unsigned long long *stats, int k, unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (wave_leader() && v) atomicAdd(&stats[k * NSLOT + wave_slot()], (unsigned long long)v);
}

PD void stat_max32(unsigned long long *stats, int k, unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    if (wave_leader() && v) atomicMax(&stats[k * NSLOT + wave_slot()], (unsigned long long)v);
}

// up to four small counters (k < 0: unused) in one wave reduction: 16-bit fields of one
// 64-bit sum, which cannot carry into each other while every lane's value is below 1024;
// otherwise (never in practice) one reduction per counter
PD void stat_add4(unsigned long long *stats, int k0, unsigned a0, int k1, unsigned a1, int k2,
                  unsigned a2, int k3, unsigned a3)
{
    if (__any(a0 >= 1024u || a1 >= 1024u || a2 >= 1024u || a3 >= 1024u)) {
        if (k0 >= 0) stat_add(stats, k0, a0);
        if (k1 >= 0) stat_add(stats, k1, a1);
        if (k2 >= 0) stat_add(stats, k2, a2);
        if (k3 >= 0) stat_add(stats, k3, a3);
        return;
    }
    unsigned long long v = (unsigned long long)a0 | ((unsigned long long)a1 << 16) |
                           ((unsigned long long)a2 << 32) | ((unsigned long long)a3 << 48);
    v = wave_sum(v);
    if (wave_leader() && v) {
        const unsigned sl = wave_slot();
        const int ks[4] = {k0, k1, k2, k3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const unsigned long long x = (v >> (16 * q)) & 0xffffull;
            if (ks[q] >= 0 && x) atomicAdd(&stats[ks[q] * NSLOT + sl], x);
        }
    }
}

// rho, u, T from conserved variables (ideal gas, R = 1): rho E = C_v rho T + rho |u|^2 / 2
template <int D>
PD void prim(const double *U, int64_t n, int64_t c, double &rho, double u[2], double &T, double Cv)
{
    rho = U[c];
    const double irho = 1.0 / rho;
    double ke = 0.0;
    for (int a = 0; a < D; ++a) {
        u[a] = U[(1 + a) * n + c] * irho;
        ke += u[a] * u[a];
    }
    if (D == 1) u[1] = 0.0;
    T = (U[(1 + D) * n + c] * irho - 0.5 * ke) / Cv;
}

PD size_t vmax_at(const Params &P, int parity, int k, int copy)
{
    return ((size_t)parity * P.n_inst + k) * P.vslots + copy;
}

// largest CFL rate of the cells this wave updates, into its instance's maximum (all lanes
// of the wave call this; `bits` is a non-negative double as its bit pattern, 0 for none)
template <typename R>
PD void vmax_update(const Params &P, const State<R> &S, int parity, int k, bool has,
                    unsigned long long bits)
{
    const int k_first = __shfl(k, 0, 64);
    if (__all(k == k_first)) {
        unsigned long long m = has ? bits : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            unsigned long long w = __shfl_xor(m, o, 64);
            m = w > m ? w : m;
        }
        if (wave_leader() && m) atomicMax(S.vmax + vmax_at(P, parity, k, wave_slot() & (P.vslots - 1)), m);
    } else if (has && bits) {
        atomicMax(S.vmax + vmax_at(P, parity, k, 0), bits);
    }
}

// ---------------------------------------------------------------------------------
// dt kernel: one 64-thread block per instance
// ---------------------------------------------------------------------------------

// dt of instance k from its CFL-rate copies of parity `slot` (which the other parity's
// cell updates filled); clears the copies of the other parity. Every lane of one wave.
// The copies and the instance's failure flag are read with device-scope atomic loads: they
// were written by atomics, which act in L2, and a resident block (below) reads them again
// on the CU that may still cache the previous step's values.
template <int D, typename R>
PD void instance_dt(const Params &P, const State<R> &S, int k, int lane, double t_end, int slot)
{
    unsigned long long m = 0ull;
    for (int c = lane; c < P.vslots; c += 64) {
        unsigned long long v =
            __hip_atomic_load(S.vmax + vmax_at(P, slot, k, c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        m = v > m ? v : m;
        S.vmax[vmax_at(P, slot ^ 1, k, c)] = 0ull;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long w = __shfl_xor(m, o, 64);
        m = w > m ? w : m;
    }
    if (lane != 0) return;
    double rate = __longlong_as_double((long long)m);
    // boundary states enter through the boundary faces: their speeds bound dt as well
    double dxa = S.dxk ? S.dxk[k] : P.dx;
    rate = fmax(rate, P.bc_speed[0] / dxa);
    if (P.dim == 2) rate = fmax(rate, P.bc_speed[1] / P.dy);
    double t = S.t[k];
    double dt = P.cfl / rate;
    const int failed = __hip_atomic_load(S.inst_err + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(rate > 0.0) || failed) dt = 0.0; // a failed instance stays frozen
    if (t + dt > t_end) dt = t_end - t;
    if (!(dt > 0.0)) dt = 0.0;
    S.tstart[k] = t;
    S.dt[k] = dt;
    S.t[k] = t + dt;
}

template <int D, typename R>
__global__ __launch_bounds__(64) void dt_kernel(Params P, State<R> S, double t_end, int slot)
{
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    if (k == 0 && S.tail_count)
        for (int c = lane; c < 2 * NSLOT; c += 64) S.tail_count[c] = 0;
    if (k == 0 && S.seed_count)
        for (int c = lane; c < NSLOT; c += 64) S.seed_count[c] = 0;
    instance_dt<D, R>(P, S, k, lane, t_end, slot);
}

// ---------------------------------------------------------------------------------
// boundary mapping and the phi-bar-plus record of one (possibly ghost) cell
// ---------------------------------------------------------------------------------

struct CellRef {
    int64_t src;   // source cell index, or -1 for a fixed state
    int mx, my;    // mirror flags
    int fside;     // side whose fixed state applies (src < 0)
    int falt;      // 0: bc_state of that side, 1: bc_alt
};

PD double xcen(const Params &P, int i) { return P.x0 + (i + 0.5) * P.dx; }
PD double ycen(const Params &P, int j) { return P.y0 + (j + 0.5) * P.dy; }

// rule of one side along one axis; g = ghost coordinate, n = cells along the axis.
// returns the source coordinate, or -1 with (fside, falt) naming the fixed state.
// (No pointer into the by-value kernel argument is formed: that would force a private
// copy of the whole parameter block.)
PD int side_rule(const Params &P, int side, int g, int n, double tpos, double xc_, double yc_,
                 double t, int &mirror, int &fside, int &falt)
{
    int kind = P.bc[side];
    if (kind == BC_SPLIT) kind = (tpos < P.bc_param[side][0]) ? BC_FIXED : BC_REFLECT;
    switch (kind) {
    case BC_PERIODIC: return (g < 0) ? g + n : g - n;
    case BC_OUTFLOW: return (g < 0) ? 0 : n - 1;
    case BC_REFLECT: mirror ^= 1; return (g < 0) ? (-1 - g) : (2 * n - 1 - g);
    case BC_FIXED: fside = side; falt = 0; return -1;
    case BC_FIXED_WINDOW:
        fside = side;
        falt = (tpos >= P.bc_param[side][0] && tpos <= P.bc_param[side][1]) ? 1 : 0;
        return -1;
    default: { // moving shock
        double xs = P.bc_param[side][0] + P.bc_param[side][1] * (yc_ + P.bc_param[side][2] * t);
        fside = side;
        falt = (xc_ < xs) ? 0 : 1;
        return -1;
    }
    }
}

// 2D: y rule first (every column), then x rule at the mapped row
PD CellRef map2d(const Params &P, int i, int j, double t)
{
    CellRef r{0, 0, 0, -1, 0};
    int si = i, sj = j;
    if (j < 0 || j >= P.ny) {
        int side = (j < 0) ? 2 : 3;
        sj = side_rule(P, side, j, P.ny, xcen(P, i), xcen(P, i), ycen(P, j), t, r.my, r.fside, r.falt);
        if (sj < 0) {
            r.src = -1;
            return r;
        }
    }
    if (i < 0 || i >= P.nx) {
        int side = (i < 0) ? 0 : 1;
        si = side_rule(P, side, i, P.nx, ycen(P, sj), xcen(P, i), ycen(P, sj), t, r.mx, r.fside, r.falt);
        if (si < 0) {
            r.src = -1;
            return r;
        }
    }
    r.src = (int64_t)si + (int64_t)P.nx * sj;
    return r;
}

// 2D population state (LAY = 1): the 16 f and 16 g populations of each cell in its own
// co-moving frame, node i = ix + 4 iy, one plane each (f planes 0..15, g planes 16..31).
// They are the same information as the 12 Hermite coefficients of the default layout (a
// change of basis, exact with the Gauss-Hermite nodes); these convert between the two.
constexpr int NPOP2 = 32;

template <typename R>
PD R inv_weight2(int i)
{
    const int ix = i & 3, iy = i >> 2;
    const double wx = (ix == 1 || ix == 2) ? Lat<double>::wa : Lat<double>::wb;
    const double wy = (iy == 1 || iy == 2) ? Lat<double>::wa : Lat<double>::wb;
    return (R)(1.0 / (wx * wy));
}

template <typename R>
PD R weight2(int i)
{
    return weight1<R>(i & 3) * weight1<R>(i >> 2);
}

// f's coefficients h20 h11 h02 h30 h21 h12 h03 and g's h10 h01 h20 h11 h02 of cell c
template <typename R>
PD void coef_from_pops_2d(const R *Pp, int64_t n, int64_t c, R fh[7], R gh[5])
{
    R p[16], mu[10], h[10];
#pragma unroll
    for (int i = 0; i < 16; ++i) p[i] = Pp[i * n + c] * inv_weight2<R>(i);
    moments_2d(p, mu, 10);
    mu2h_2d(mu, h, 10);
#pragma unroll
    for (int k = 0; k < 7; ++k) fh[k] = h[3 + k];
#pragma unroll
    for (int i = 0; i < 16; ++i) p[i] = Pp[(16 + i) * n + c] * inv_weight2<R>(i);
    moments_2d(p, mu, 6);
    mu2h_2d(mu, h, 6);
#pragma unroll
    for (int k = 0; k < 5; ++k) gh[k] = h[1 + k];
}

// the 32 populations of cell c from its coefficients: f from (rho, 0, 0, fh), g from
// (b0, gh) with g's zeroth coefficient b0 = (C_v - 1) rho T - T (h20 + h02) (the energy)
template <typename R>
PD void pops_from_coef_2d(R *Pp, int64_t n, int64_t c, R rho, R b0, const R fh[7], const R gh[5])
{
    R h[10] = {rho, R(0), R(0), fh[0], fh[1], fh[2], fh[3], fh[4], fh[5], fh[6]};
    R p[16];
    eval_2d(h, p, 3);
#pragma unroll
    for (int i = 0; i < 16; ++i) Pp[i * n + c] = weight2<R>(i) * p[i];
    R hg[10] = {b0, gh[0], gh[1], gh[2], gh[3], gh[4], R(0), R(0), R(0), R(0)};
    eval_2d(hg, p, 2);
#pragma unroll
    for (int i = 0; i < 16; ++i) Pp[(16 + i) * n + c] = weight2<R>(i) * p[i];
}

// phi-bar-plus of one cell into an LDS record (Sec. III.B.3): phi+ = A f~ + B f_eq with
// A = (2 - eps/2)/(2 + eps), B = (3 eps/2)/(2 + eps), eps = dt p / mu; f_eq = rho W_i
// and g_eq = (C_v - D/2) rho T W_i in the co-moving frame (Sec. II.B).
template <int D, typename R, int LAY = 0>
PD void plus_record(const Params &P, const State<R> &S, const CellRef &c, double dt, R *out,
                    int NT, int slot)
{
    double rho, u[2], T;
    R fh[7] = {0, 0, 0, 0, 0, 0, 0}, gh[5] = {0, 0, 0, 0, 0};
    const int nfh = (D == 1) ? 2 : 7, ngh = (D == 1) ? 2 : 5;
    if (c.src < 0) {
        double st[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) st[q] = c.falt ? P.bc_alt[c.fside][q] : P.bc_state[c.fside][q];
        rho = st[0];
        u[0] = st[1];
        u[1] = (D == 2) ? st[2] : 0.0;
        T = st[3] / st[0];
    } else {
        prim<D>(S.U, P.ncell, c.src, rho, u, T, P.Cv);
        if constexpr (D == 2 && LAY == 1) {
            coef_from_pops_2d(S.H, P.ncell, c.src, fh, gh);
        } else {
#pragma unroll
            for (int k = 0; k < nfh; ++k) fh[k] = S.H[k * P.ncell + c.src];
#pragma unroll
            for (int k = 0; k < ngh; ++k) gh[k] = S.H[(nfh + k) * P.ncell + c.src];
        }
        if (D == 1) {
            if (c.mx) {
                u[0] = -u[0];
                fh[1] = -fh[1];
                gh[0] = -gh[0];
            }
        } else {
            if (c.mx) { // odd x degree flips: f h11 h30 h12, g h10 h11
                u[0] = -u[0];
                fh[1] = -fh[1];
                fh[3] = -fh[3];
                fh[5] = -fh[5];
                gh[0] = -gh[0];
                gh[3] = -gh[3];
            }
            if (c.my) { // odd y degree flips: f h11 h21 h03, g h01 h11
                u[1] = -u[1];
                fh[1] = -fh[1];
                fh[4] = -fh[4];
                fh[6] = -fh[6];
                gh[1] = -gh[1];
                gh[3] = -gh[3];
            }
        }
    }
    const double eps = dt * rho * T / P.mu;
    const double i2e = 1.0 / (2.0 + eps);
    const double Ap = (2.0 - 0.5 * eps) * i2e, Bp = 1.5 * eps * i2e;
    const double geq = (P.Cv - 0.5 * D) * rho * T;
    // g~'s zeroth coefficient from the energy: rho E = rho|u|^2/2 + T(tr h2 + D rho/2) + b0
    double trh2 = (D == 1) ? (double)fh[0] : (double)fh[0] + (double)fh[2];
    double b0 = geq - T * trh2;
    if (D == 1) {
        out[0 * NT] = (R)u[0];
        out[1 * NT] = (R)sqrt(T);
        out[2 * NT] = (R)T;
        out[3 * NT] = (R)rho;
        out[4 * NT] = (R)(Ap * fh[0]);
        out[5 * NT] = (R)(Ap * fh[1]);
        out[6 * NT] = (R)(Ap * b0 + Bp * geq);
        out[7 * NT] = (R)(Ap * gh[0]);
        out[8 * NT] = (R)(Ap * gh[1]);
    } else {
        out[0 * NT] = (R)u[0];
        out[1 * NT] = (R)u[1];
        out[2 * NT] = (R)sqrt(T);
        out[3 * NT] = (R)rho;
        // coefficients in the scaled form of q2mu_2d (times a! b!)
        constexpr double fq[7] = {2.0, 1.0, 2.0, 6.0, 2.0, 2.0, 6.0}, gq[5] = {1.0, 1.0, 2.0, 1.0, 2.0};
        for (int k = 0; k < 7; ++k) out[(4 + k) * NT] = (R)(Ap * fq[k] * fh[k]);
        out[11 * NT] = (R)(Ap * b0 + Bp * geq);
        for (int k = 0; k < 5; ++k) out[(12 + k) * NT] = (R)(Ap * gq[k] * gh[k]);
        out[17 * NT] = (R)T;
    }
    (void)slot;
}

// ---------------------------------------------------------------------------------
// stencil populations in the current face frame
// ---------------------------------------------------------------------------------

// reduced populations of stencil cell c (LDS record) in frame (u, s); f (NC = full
// degree 3) or g (degree 2)
template <typename R, bool G>
PD void cell_pops_1d(const R *L, int NT, int c, R u, R inv_s, R p[4])
{
    R r = L[1 * NT + c] * inv_s, d = (L[c] - u) * inv_s;
    R h[4], mu[4];
    if (!G) {
        h[0] = L[3 * NT + c];
        h[1] = R(0);
        h[2] = L[4 * NT + c];
        h[3] = L[5 * NT + c];
    } else {
        h[0] = L[6 * NT + c];
        h[1] = L[7 * NT + c];
        h[2] = L[8 * NT + c];
        h[3] = R(0);
    }
    h2mu_1d(h, mu);
    shift_1d(mu, r, d, G ? 3 : 4);
    mu2h_1d(mu, h);
    eval_1d(h, p, G ? 2 : 3);
}

// The 2D records hold the coefficients in the scaled form q (see q2mu_2d); the transform
// into the face frame and the evaluation work on that form. REG = 1: the f populations of
// the alternative regularization (eq_fast_2d), the g populations unchanged.
template <typename R, bool G, int REG = 0>
PD void cell_pops_2d(const R *L, int NT, int c, R ux, R uy, R inv_s, R p[16])
{
    R r = L[2 * NT + c] * inv_s, dx = (L[c] - ux) * inv_s, dy = (L[NT + c] - uy) * inv_s;
    R q[10], mu[10];
    if (!G) {
        q[0] = L[3 * NT + c];
        q[1] = R(0);
        q[2] = R(0);
#pragma unroll
        for (int k = 0; k < 7; ++k) q[3 + k] = L[(4 + k) * NT + c];
        q2mu_2d(q, mu, 10);
        shift_2d(mu, r, dx, dy, 10);
        mu2q_2d(mu, q, 10);
        if (REG) {
            R qf[6];
            eq_fast_2d(q, qf);
            eval_q16_2d(q, qf, p);
        } else {
            eval_q_2d(q, p, 3);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = L[(11 + k) * NT + c];
        q2mu_2d(q, mu, 6);
        shift_2d(mu, r, dx, dy, 6);
        mu2q_2d(mu, q, 6);
        eval_q_2d(q, p, 2);
    }
}

// the populations of stencil cell c in the node columns `cols` (wave-uniform) only
template <typename R, bool G, int AXIS, int REG = 0>
PD void cell_cols_2d(const R *L, int NT, int c, R ux, R uy, R inv_s, int cols, R p[16])
{
    R r = L[2 * NT + c] * inv_s, dx = (L[c] - ux) * inv_s, dy = (L[NT + c] - uy) * inv_s;
    R q[10], mu[10];
    if (!G) {
        q[0] = L[3 * NT + c];
        q[1] = R(0);
        q[2] = R(0);
#pragma unroll
        for (int k = 0; k < 7; ++k) q[3 + k] = L[(4 + k) * NT + c];
        q2mu_2d(q, mu, 10);
        shift_2d(mu, r, dx, dy, 10);
        mu2q_2d(mu, q, 10);
        if (REG) {
            R qf[6];
            eq_fast_2d(q, qf);
            eval_q16_cols_2d<R, AXIS>(q, qf, cols, p);
        } else {
            eval_q_cols_2d<R, AXIS>(q, cols, p, 3);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) q[k] = L[(11 + k) * NT + c];
        q2mu_2d(q, mu, 6);
        shift_2d(mu, r, dx, dy, 6);
        mu2q_2d(mu, q, 6);
        eval_q_cols_2d<R, AXIS>(q, cols, p, 2);
    }
}

// MUSCL reconstruction at the departure points, 1D. idx: L, R, L-1, R+1.
// Returns the reduced populations phi-bar_i / W_i at the face.
template <typename R, bool G>
PD void recon_1d(const R *L, int NT, const int idx[4], R u, R s, R inv_s, R hdx, int lim,
                 R out[4])
{
    R PL[4], PR[4], T[4], A[4];
    cell_pops_1d<R, G>(L, NT, idx[0], u, inv_s, PL);
    cell_pops_1d<R, G>(L, NT, idx[1], u, inv_s, PR);
    cell_pops_1d<R, G>(L, NT, idx[2], u, inv_s, T);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        R v = s * node<R>(i) + u;
        A[i] = (v >= R(0)) ? PL[i] - T[i] : PR[i] - PL[i];
    }
    cell_pops_1d<R, G>(L, NT, idx[3], u, inv_s, T);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        R v = s * node<R>(i) + u;
        bool up = v >= R(0);
        R B = up ? PR[i] - PL[i] : T[i] - PR[i];
        // slope from limit_part, offset scaled by limit_scale (bitwise the same product)
        const R sc = R(limit_scale(lim));
        R sl = limit_part(A[i], B, lim);
        R off = (up ? R(0.5) * sc : R(-0.5) * sc) - v * (hdx * sc);
        out[i] = (up ? PL[i] : PR[i]) + off * sl;
    }
}

// 2D, face normal along AXIS, all 16 populations at once (FP32 records). idx: L, R, L-n,
// R+n, L-t, L+t, R-t, R+t.
// SUB: every lane of the wave takes the two negative normal node columns from the R side
// and the two positive ones from the L side (|normal frame velocity| below s*ca, the usual
// case); the side cells of the stencil are then evaluated in the two columns they feed only.
template <typename R, bool G, int AXIS, bool SUB, int REG = 0>
PD void recon_2d_whole(const R *L, int NT, const int idx[8], R ux, R uy, R s, R inv_s, R hdn, R hdt,
                 int lim, R M[10])
{
    R PL[16], PR[16], T[16], A[16], out[16];
    const R un = AXIS ? uy : ux, ut = AXIS ? ux : uy;
    bool upn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) upn[k] = fma(s, node<R>(k), un) >= R(0);
    auto nk = [](int i) { return AXIS ? (i >> 2) : (i & 3); };
    auto tk = [](int i) { return AXIS ? (i & 3) : (i >> 2); };
    // the SUB and full forms give bitwise the same values in every lane (the choice between
    // them depends on the other lanes of the wave): products that feed sums are written as
    // explicit fma, so the compiler's contraction choices cannot differ between the two
    if (SUB) {
#pragma unroll
        for (int k = 0; k < 4; ++k) upn[k] = k >= 2;
    }
    constexpr int cup = SUB ? 0xC : 0xF, cdn = SUB ? 0x3 : 0xF;
    const R sc = R(limit_scale(lim)); // slopes come from limit_part
    cell_pops_2d<R, G, REG>(L, NT, idx[0], ux, uy, inv_s, PL);
    __builtin_amdgcn_sched_barrier(0);
    cell_pops_2d<R, G, REG>(L, NT, idx[1], ux, uy, inv_s, PR);
    __builtin_amdgcn_sched_barrier(0);
    cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[2], ux, uy, inv_s, cup, T);
#pragma unroll
    for (int i = 0; i < 16; ++i) A[i] = upn[nk(i)] ? PL[i] - T[i] : PR[i] - PL[i];
    __builtin_amdgcn_sched_barrier(0);
    cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[3], ux, uy, inv_s, cdn, T);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const bool up = upn[nk(i)];
        R vn = fma(s, node<R>(nk(i)), un);
        R B = up ? PR[i] - PL[i] : T[i] - PR[i];
        R sl = limit_part(A[i], B, lim);
        R off = fma(-vn, hdn * sc, up ? R(0.5) * sc : R(-0.5) * sc);
        R pu = up ? PL[i] : PR[i];
        out[i] = fma(off, sl, pu);
        PL[i] = pu; // upwind value, kept for the tangential slope
    }
    // tangential slope of the upwind cell
    __builtin_amdgcn_sched_barrier(0);
    cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[4], ux, uy, inv_s, cup, T);
#pragma unroll
    for (int i = 0; i < 16; ++i) A[i] = PL[i] - T[i];
    __builtin_amdgcn_sched_barrier(0);
    cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[6], ux, uy, inv_s, cdn, T);
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (!upn[nk(i)]) A[i] = PL[i] - T[i];
    __builtin_amdgcn_sched_barrier(0);
    cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[5], ux, uy, inv_s, cup, T);
#pragma unroll
    for (int i = 0; i < 16; ++i) PR[i] = T[i] - PL[i];
    __builtin_amdgcn_sched_barrier(0);
    cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[7], ux, uy, inv_s, cdn, T);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        R B = upn[nk(i)] ? PR[i] : T[i] - PL[i];
        R sl = limit_part(A[i], B, lim);
        R vt = fma(s, node<R>(tk(i)), ut);
        A[i] = fma(-vt * (hdt * sc), sl, out[i]);
    }
    moments_2d(A, M, G ? 6 : 10);
}

// 2D, face normal along AXIS, half a face at a time (FP64 records). idx as recon_2d_whole.
// SUB: every lane of the wave takes the two negative normal node columns from the R side
// and the two positive ones from the L side (|normal frame velocity| below s*ca, the usual
// case); the side cells of the stencil are then evaluated in the two columns they feed only.
// The face is done half at a time (normal node columns 2, 3, then 0, 1): every stencil cell
// a half needs is transformed into the face frame again for it (L and R twice in the SUB
// form), which keeps the live set at a few arrays of 8 populations; each half's columns are
// reduced over the tangential nodes at once, and the normal stage closes the moments.
template <typename R, bool G, int AXIS, bool SUB, int REG = 0>
PD void recon_2d_halves(const R *L, int NT, const int idx[8], R ux, R uy, R s, R inv_s, R hdn, R hdt,
                 int lim, R M[10])
{
    const R un = AXIS ? uy : ux, ut = AXIS ? ux : uy;
    bool upn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) upn[k] = SUB ? (k >= 2) : (fma(s, node<R>(k), un) >= R(0));
    auto nk = [](int i) { return AXIS ? (i >> 2) : (i & 3); };
    auto tk = [](int i) { return AXIS ? (i & 3) : (i >> 2); };
    auto pi = [](int n, int t) { return AXIS ? (t + 4 * n) : (n + 4 * t); };
    // the SUB and full forms give bitwise the same values in every lane (the choice between
    // them depends on the other lanes of the wave): every population goes through the same
    // operations in both, and products that feed sums are explicit fma
    const R sc = R(limit_scale(lim)); // slopes come from limit_part
    R Rt[4][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int cols = h ? 0x3 : 0xC;
        R PL[16], PR[16], T[16], A[16], out[16];
        __builtin_amdgcn_sched_barrier(0);
        cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[0], ux, uy, inv_s, cols, PL);
        __builtin_amdgcn_sched_barrier(0);
        cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[1], ux, uy, inv_s, cols, PR);
        if (!SUB || h == 0) {
            __builtin_amdgcn_sched_barrier(0);
            cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[2], ux, uy, inv_s, cols, T);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (cols & (1 << nk(i))) A[i] = upn[nk(i)] ? PL[i] - T[i] : PR[i] - PL[i];
        if (!SUB || h == 1) {
            __builtin_amdgcn_sched_barrier(0);
            cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[3], ux, uy, inv_s, cols, T);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (!(cols & (1 << nk(i)))) continue;
            const bool up = upn[nk(i)];
            R vn = fma(s, node<R>(nk(i)), un);
            R B = up ? PR[i] - PL[i] : T[i] - PR[i];
            R sl = limit_part(A[i], B, lim);
            R off = fma(-vn, hdn * sc, up ? R(0.5) * sc : R(-0.5) * sc);
            R pu = up ? PL[i] : PR[i];
            out[i] = fma(off, sl, pu);
            PL[i] = pu; // upwind value, kept for the tangential slope
        }
        // tangential slope of the upwind cell: backward neighbour L-t or R-t, forward L+t or R+t
        if (!SUB || h == 0) {
            __builtin_amdgcn_sched_barrier(0);
            cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[4], ux, uy, inv_s, cols, T);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (cols & (1 << nk(i))) A[i] = PL[i] - T[i];
        }
        if (!SUB || h == 1) {
            __builtin_amdgcn_sched_barrier(0);
            cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[6], ux, uy, inv_s, cols, T);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if ((cols & (1 << nk(i))) && !upn[nk(i)]) A[i] = PL[i] - T[i];
        }
        if (!SUB || h == 0) {
            __builtin_amdgcn_sched_barrier(0);
            cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[5], ux, uy, inv_s, cols, T);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (cols & (1 << nk(i))) PR[i] = T[i] - PL[i];
        }
        if (!SUB || h == 1) {
            __builtin_amdgcn_sched_barrier(0);
            cell_cols_2d<R, G, AXIS, REG>(L, NT, idx[7], ux, uy, inv_s, cols, T);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (!(cols & (1 << nk(i)))) continue;
            R B = upn[nk(i)] ? PR[i] : T[i] - PL[i];
            R sl = limit_part(A[i], B, lim);
            R vt = fma(s, node<R>(tk(i)), ut);
            out[i] = fma(-vt * (hdt * sc), sl, out[i]);
        }
#pragma unroll
        for (int n = 0; n < 4; ++n)
            if (cols & (1 << n)) tan_sums(out[pi(n, 0)], out[pi(n, 1)], out[pi(n, 2)], out[pi(n, 3)], Rt[n]);
    }
    normal_sums<R, AXIS>(Rt, M, G ? 6 : 10);
}

// The reconstruction of one face iteration. FP64: half a face at a time, which holds the
// FP64 face kernel at 247 registers (2 waves per SIMD without spills, where the whole-face
// form needs about 282 and spills); FP32: the whole face, whose one transform of L and R
// per iteration is cheaper there (142 against 161 registers, both 3 waves per SIMD, and the
// halves' second transforms made the FP32 kernel 7% slower).
template <typename R, bool G, int AXIS, bool SUB, int REG = 0>
PD void recon_2d(const R *L, int NT, const int idx[8], R ux, R uy, R s, R inv_s, R hdn, R hdt,
                 int lim, R M[10])
{
    if constexpr (sizeof(R) == 8)
        recon_2d_halves<R, G, AXIS, SUB, REG>(L, NT, idx, ux, uy, s, inv_s, hdn, hdt, lim, M);
    else
        recon_2d_whole<R, G, AXIS, SUB, REG>(L, NT, idx, ux, uy, s, inv_s, hdn, hdt, lim, M);
}

// ---------------------------------------------------------------------------------
// face finalization: moments of phi-bar in frame `last` -> phi in the final frame
// ---------------------------------------------------------------------------------

// writes the face state: frame, f coefficients (degree 3) and g coefficients (degree 2)
// of phi = (phi-bar + (eps/4) phi_eq) / (1 + eps/4), phi_eq the co-moving equilibrium of the
// final frame (Sec. III.B.3), eps = dt p_b / mu.
template <int D, typename R>
PD void face_write(const Params &P, const State<R> &S, int64_t f, R *mf, R *mg, const R *ul,
                   R sl, const R *uf, R Tf, bool has_frame, double dt)
{
    const int64_t nf = P.nface;
    R sf = sqrt(Tf);
    if (D == 1) {
        R h[4], hg[4];
        if (has_frame) {
            R inv = frcp(sf);
            shift_1d(mf, sl * inv, (ul[0] - uf[0]) * inv, 4);
            shift_1d(mg, sl * inv, (ul[0] - uf[0]) * inv, 3);
        }
        mu2h_1d(mf, h);
        mg[3] = R(0);
        mu2h_1d(mg, hg);
        R rho = h[0];
        double eps = has_frame ? dt * (double)rho * (double)Tf / P.mu : 0.0;
        R c = (R)(1.0 / (1.0 + 0.25 * eps));
        R e4 = (R)(0.25 * eps);
        S.F[0 * nf + f] = uf[0];
        S.F[1 * nf + f] = Tf;
        S.F[2 * nf + f] = rho;
        S.F[3 * nf + f] = h[1] * c;
        S.F[4 * nf + f] = h[2] * c;
        S.F[5 * nf + f] = h[3] * c;
        S.F[6 * nf + f] = (hg[0] + e4 * (R)(P.Cv - 0.5) * rho * Tf) * c;
        S.F[7 * nf + f] = hg[1] * c;
        S.F[8 * nf + f] = hg[2] * c;
    } else {
        R h[10], hg[10];
        if (has_frame) {
            R inv = frcp(sf);
            R r = sl * inv, dx = (ul[0] - uf[0]) * inv, dy = (ul[1] - uf[1]) * inv;
            shift_2d(mf, r, dx, dy, 10);
            shift_2d(mg, r, dx, dy, 6);
        }
        mu2h_2d(mf, h, 10);
        mu2h_2d(mg, hg, 6);
        R rho = h[0];
        R c, e4;
        if constexpr (sizeof(R) == 4) {
            const R eps = has_frame ? (R)(dt / P.mu) * rho * Tf : R(0);
            e4 = R(0.25) * eps;
            c = frcp(R(1) + e4);
        } else {
            double eps = has_frame ? dt * (double)rho * (double)Tf / P.mu : 0.0;
            c = (R)(1.0 / (1.0 + 0.25 * eps));
            e4 = (R)(0.25 * eps);
        }
        S.F[0 * nf + f] = uf[0];
        S.F[1 * nf + f] = uf[1];
        S.F[2 * nf + f] = Tf;
        S.F[3 * nf + f] = rho;
#pragma unroll
        for (int k = 1; k < 10; ++k) S.F[(3 + k) * nf + f] = h[k] * c;
        S.F[13 * nf + f] = (hg[0] + e4 * (R)(P.Cv - 1.0) * rho * Tf) * c;
#pragma unroll
        for (int k = 1; k < 6; ++k) S.F[(13 + k) * nf + f] = hg[k] * c;
    }
}

// mean frame of two cells' conserved variables (seed of the first step, restart frame):
// with S = rho_a + rho_b, u = (rho_a u_a + rho_b u_b) / S and, from the mean energy,
// T = (rho_a T_a + rho_b T_b) / S + rho_a rho_b |u_a - u_b|^2 / (2 C_v S^2) -- the same value
// as (E/rho - |u|^2/2)/C_v of the mean conserved variables, without its cancellation, so
// it is evaluated in the record precision
template <int D, typename R>
PD void mean_frame(const R *L, int NT, int a, int b, const Params &P, R u[2], R &T)
{
    const int sT = (D == 1) ? 2 : 17, sr = 3;
    const R ra = L[sr * NT + a], rb = L[sr * NT + b];
    const R Sm = ra + rb, iS = (sizeof(R) == 4) ? frcp(Sm) : R(1) / Sm;
    const R wa = ra * iS, wb = rb * iS;
    R du2 = R(0);
    for (int q = 0; q < D; ++q) {
        const R ua = L[q * NT + a], ub = L[q * NT + b];
        u[q] = wa * ua + wb * ub;
        du2 += (ua - ub) * (ua - ub);
    }
    if (D == 1) u[1] = R(0);
    T = wa * L[sT * NT + a] + wb * L[sT * NT + b] + wa * wb * du2 * (R)(0.5 / P.Cv);
}

// first-order upwind state from each neighbour's own frame (fallback), as raw moments
// in frame (um, sm)
template <typename R, bool G>
PD void own_half_1d(const R *L, int NT, int c, bool right, R um, R inv_sm, R mu[4])
{
    R u = L[c], s = L[NT + c];
    R h[4], p[4];
    if (!G) {
        h[0] = L[3 * NT + c];
        h[1] = R(0);
        h[2] = L[4 * NT + c];
        h[3] = L[5 * NT + c];
    } else {
        h[0] = L[6 * NT + c];
        h[1] = L[7 * NT + c];
        h[2] = L[8 * NT + c];
        h[3] = R(0);
    }
    eval_1d(h, p, G ? 2 : 3);
    for (int i = 0; i < 4; ++i) {
        R v = s * node<R>(i) + u;
        bool take = right ? (v < R(0)) : (v >= R(0));
        if (!take) p[i] = R(0);
    }
    moments_1d(p, mu, 4);
    shift_1d(mu, s * inv_sm, (u - um) * inv_sm, 4);
}

template <typename R, bool G, int AXIS, int REG = 0>
PD void own_half_2d(const R *L, int NT, int c, bool right, R umx, R umy, R inv_sm, R mu[10])
{
    R ux = L[c], uy = L[NT + c], s = L[2 * NT + c];
    R q[10], p[16]; // scaled coefficients of the record (see q2mu_2d)
    if (!G) {
        q[0] = L[3 * NT + c];
        q[1] = R(0);
        q[2] = R(0);
        for (int k = 0; k < 7; ++k) q[3 + k] = L[(4 + k) * NT + c];
        if (REG) {
            R qf[6];
            eq_fast_2d(q, qf);
            eval_q16_2d(q, qf, p);
        } else {
            eval_q_2d(q, p, 3);
        }
    } else {
        for (int k = 0; k < 6; ++k) q[k] = L[(11 + k) * NT + c];
        eval_q_2d(q, p, 2);
    }
    const R un = AXIS ? uy : ux;
    for (int i = 0; i < 16; ++i) {
        R v = s * node<R>(AXIS ? (i >> 2) : (i & 3)) + un;
        bool take = right ? (v < R(0)) : (v >= R(0));
        if (!take) p[i] = R(0);
    }
    moments_2d(p, mu, 10);
    shift_2d(mu, s * inv_sm, (ux - umx) * inv_sm, (uy - umy) * inv_sm, 10);
}

// ---------------------------------------------------------------------------------
// the face iteration (Sec. III.B.3)
// ---------------------------------------------------------------------------------

// Frame-update arithmetic: FP32 uses the hardware reciprocal estimates (about 1 ulp), FP64
// the correctly rounded operations in the oracle's form.
template <typename R>
PD void frame_scale(R T, R &s, R &inv_s)
{
    if constexpr (sizeof(R) == 4) {
        inv_s = frsq(T);
        s = T * inv_s;
    } else {
        s = sqrt(T);
        inv_s = R(1) / s;
    }
}

template <typename R>
PD R temperature(R rhoe, R rho, R irho, double Cv)
{
    if constexpr (sizeof(R) == 4)
        return rhoe * irho * (R)(1.0 / Cv);
    else
        return rhoe / ((R)Cv * rho);
}

// relative change |a - b| / T
template <typename R>
PD R rel(R a, R b, R T, R iT)
{
    if constexpr (sizeof(R) == 4)
        return fabs(a - b) * iT;
    else
        return fabs(a - b) / T;
}

struct FaceCount {
    unsigned long long iters, nonconv, fallback, depout, itmax;
    unsigned long long tail_faces = 0, tail_iters = 0; // faces finished by the tail kernel
};

// 1D face f with LDS stencil indices idx = {L, R, L-1, R+1}
template <typename R, int LIM>
PD void face_1d(const Params &P, const State<R> &S, const R *L, int NT, const int idx[4], int64_t f,
                double dt, double dx, FaceCount &cnt)
{
    const R hdx = (R)(0.5 * dt / dx);
    const int64_t nf = P.nface;
    R u[2] = {S.F[0 * nf + f], R(0)}, T = S.F[1 * nf + f];
    R mu_m[2];
    R T_m;
    mean_frame<1, R>(L, NT, idx[0], idx[1], P, mu_m, T_m);
    bool restarted = false;
    if (!(T > R(0))) {
        u[0] = mu_m[0];
        T = T_m;
        restarted = true;
    }
    R mf[4], mg[4], ul[2] = {u[0], R(0)}, sl = sqrt(T);
    R upp = u[0], Tpp = T; // frame two iterations back
    bool have_pp = false;
    int it = 0;
    bool conv = false, failed = false;
    while (it < P.max_iter) {
        ++it;
        R s, inv_s;
        frame_scale(T, s, inv_s);
        R qf[4], qg[4];
        recon_1d<R, false>(L, NT, idx, u[0], s, inv_s, hdx, LIM, qf);
        recon_1d<R, true>(L, NT, idx, u[0], s, inv_s, hdx, LIM, qg);
        moments_1d(qf, mf, 4);
        moments_1d(qg, mg, 3);
        R rho = mf[0];
        // FP32: hardware reciprocal estimates; FP64: correctly rounded divisions
        R irho = R(0), du, rhoe;
        if constexpr (sizeof(R) == 4) {
            irho = frcp(rho);
            du = s * mf[1] * irho;
            rhoe = R(0.5) * s * s * (mf[2] - mf[1] * mf[1] * irho) + mg[0];
        } else {
            du = s * mf[1] / rho;
            rhoe = R(0.5) * s * s * (mf[2] - mf[1] * mf[1] / rho) + mg[0];
        }
        R Tn = temperature(rhoe, rho, irho, P.Cv);
        if (!(rho > R(0)) || !(Tn > R(0)) || !isfinite(Tn) || !isfinite(du)) {
            if (!restarted) {
                restarted = true;
                u[0] = mu_m[0];
                T = T_m;
                have_pp = false;
                continue;
            }
            failed = true;
            break;
        }
        R un = u[0] + du;
        R delta, delta2;
        if constexpr (sizeof(R) == 4) {
            const R isq = frsq(Tn), iTn = isq * isq;
            delta = fmax(fabs(du) * isq, rel(Tn, T, Tn, iTn));
            delta2 = fmax(fabs(un - upp) * isq, rel(Tn, Tpp, Tn, iTn));
        } else {
            delta = fmax(fabs(du) / sqrt(Tn), fabs(Tn - T) / Tn);
            delta2 = fmax(fabs(un - upp) / sqrt(Tn), fabs(Tn - Tpp) / Tn);
        }
        upp = u[0];
        Tpp = T;
        ul[0] = u[0];
        sl = s;
        u[0] = un;
        T = Tn;
        if (delta <= (R)P.tol) {
            conv = true;
            break;
        }
        // an iteration that returns to the frame two iterations back oscillates: stop
        if (have_pp && delta2 <= R(1e-2) * delta) break;
        have_pp = true;
    }
    bool has_frame = true;
    if (failed || !conv) {
        // first-order upwind state from the neighbours' own frames
        R inv_sm = R(1) / sqrt(T_m);
        R a[4], b[4];
        own_half_1d<R, false>(L, NT, idx[0], false, mu_m[0], inv_sm, a);
        own_half_1d<R, false>(L, NT, idx[1], true, mu_m[0], inv_sm, b);
        for (int k = 0; k < 4; ++k) mf[k] = a[k] + b[k];
        own_half_1d<R, true>(L, NT, idx[0], false, mu_m[0], inv_sm, a);
        own_half_1d<R, true>(L, NT, idx[1], true, mu_m[0], inv_sm, b);
        for (int k = 0; k < 4; ++k) mg[k] = a[k] + b[k];
        R sm = sqrt(T_m);
        R rho = mf[0];
        R du = sm * mf[1] / rho;
        R Tn = (R(0.5) * sm * sm * (mf[2] - mf[1] * mf[1] / rho) + mg[0]) / ((R)P.Cv * rho);
        ul[0] = mu_m[0];
        sl = sm;
        if (rho > R(0) && Tn > R(0) && isfinite(Tn) && isfinite(du)) {
            u[0] = mu_m[0] + du;
            T = Tn;
        } else {
            has_frame = false;
            u[0] = mu_m[0];
            T = T_m;
        }
        cnt.fallback += 1;
    }
    {
        R s = sqrt(T);
        R v0 = s * node<R>(3) + fabs(u[0]);
        if (v0 * (R)(0.5 * dt) > (R)(0.5 * dx)) cnt.depout += 1;
    }
    if (!conv) cnt.nonconv += 1;
    cnt.iters += it;
    if ((unsigned long long)it > cnt.itmax) cnt.itmax = it;
    face_write<1, R>(P, S, f, mf, mg, ul, sl, u, T, has_frame, dt);
    S.fiter[f] = it | ((conv ? 0 : 1) << 16) | ((failed ? 1 : 0) << 17);
}

// cell (ci, cj) of stencil slot q (L, R, L-n, R+n, L-t, L+t, R-t, R+t) of face f
template <int AXIS>
PD void tail_cell(const Params &P, int64_t f, int q, int &ci, int &cj)
{
    int i, j; // the face's upper/right cell R
    if (AXIS == 0) {
        i = (int)(f % (P.nx + 1));
        j = (int)(f / (P.nx + 1));
    } else {
        const int64_t g = f - P.nfx;
        i = (int)(g % P.nx);
        j = (int)(g / P.nx);
    }
    const int a = (q == 1 || q >= 6) ? 1 : (q == 2 ? -1 : (q == 3 ? 2 : 0)); // normal, from L
    const int b = (q == 4 || q == 6) ? -1 : ((q == 5 || q == 7) ? 1 : 0);   // tangential
    if (AXIS == 0) {
        ci = i - 1 + a;
        cj = j + b;
    } else {
        ci = i + b;
        cj = j - 1 + a;
    }
}

template <typename R, int AXIS, int LIM, int REG = 0>
PD void face_2d(const Params &P, const State<R> &S, const R *L, int NT, const int idx[2], int sn,
                int stn, int64_t f, double dt, FaceCount &cnt)
{
    const double dn = AXIS ? P.dy : P.dx, dtn = AXIS ? P.dx : P.dy;
    const R hdn = (R)(0.5 * dt / dn), hdt = (R)(0.5 * dt / dtn);
    const int64_t nf = P.nface;
    R u[2] = {S.F[0 * nf + f], S.F[1 * nf + f]}, T = S.F[2 * nf + f];
    R um[2], T_m;
    mean_frame<2, R>(L, NT, idx[0], idx[1], P, um, T_m);
    bool restarted = false;
    if (!(T > R(0))) {
        u[0] = um[0];
        u[1] = um[1];
        T = T_m;
        restarted = true;
    }
    R mf[10], mg[10], ul[2] = {u[0], u[1]}, sl = sqrt(T);
    R upp[2] = {u[0], u[1]}, Tpp = T; // frame two iterations back
    bool have_pp = false;
    int it = 0;
    bool conv = false, failed = false, stopped = false;
    const int kcap = (P.iter_split > 0 && P.iter_split < P.max_iter) ? P.iter_split : P.max_iter;
    while (it < kcap) {
        ++it;
        R s, inv_s;
        frame_scale(T, s, inv_s);
        {
            const int b0 = idx[0];
            const int sidx[8] = {b0, b0 + sn, b0 - sn, b0 + 2 * sn, b0 - stn, b0 + stn, b0 + sn - stn, b0 + sn + stn};
            const R un = AXIS ? u[1] : u[0];
            if (__all(!(fma(s, node<R>(1), un) >= R(0)) && (fma(s, node<R>(2), un) >= R(0)))) {
                recon_2d<R, false, AXIS, true, REG>(L, NT, sidx, u[0], u[1], s, inv_s, hdn, hdt, LIM, mf);
                recon_2d<R, true, AXIS, true>(L, NT, sidx, u[0], u[1], s, inv_s, hdn, hdt, LIM, mg);
            } else {
                recon_2d<R, false, AXIS, false, REG>(L, NT, sidx, u[0], u[1], s, inv_s, hdn, hdt, LIM, mf);
                recon_2d<R, true, AXIS, false>(L, NT, sidx, u[0], u[1], s, inv_s, hdn, hdt, LIM, mg);
            }
        }
        R rho = mf[0];
        R irho = (sizeof(R) == 4) ? frcp(rho) : R(1) / rho;
        R dux = s * mf[1] * irho, duy = s * mf[2] * irho;
        R rhoe = R(0.5) * s * s * (mf[3] + mf[5] - (mf[1] * mf[1] + mf[2] * mf[2]) * irho) + mg[0];
        R Tn = temperature(rhoe, rho, irho, P.Cv);
        if (!(rho > R(0)) || !(Tn > R(0)) || !isfinite(Tn) || !isfinite(dux) || !isfinite(duy)) {
            if (!restarted) {
                restarted = true;
                u[0] = um[0];
                u[1] = um[1];
                T = T_m;
                have_pp = false;
                continue;
            }
            failed = true;
            break;
        }
        const R unx = u[0] + dux, uny = u[1] + duy;
        const R isq = (sizeof(R) == 4) ? frsq(Tn) : R(1) / sqrt(Tn), iTn = isq * isq;
        R delta = fmax(fmax(fabs(dux), fabs(duy)) * isq, rel(Tn, T, Tn, iTn));
        R delta2 = fmax(fmax(fabs(unx - upp[0]), fabs(uny - upp[1])) * isq, rel(Tn, Tpp, Tn, iTn));
        upp[0] = u[0];
        upp[1] = u[1];
        Tpp = T;
        ul[0] = u[0];
        ul[1] = u[1];
        sl = s;
        u[0] = unx;
        u[1] = uny;
        T = Tn;
        if (delta <= (R)P.tol) {
            conv = true;
            break;
        }
        // an iteration that returns to the frame two iterations back oscillates: stop
        if (have_pp && delta2 <= R(1e-2) * delta) {
            stopped = true;
            break;
        }
        have_pp = true;
    }
    if (!conv && !failed && !stopped && it < P.max_iter) {
        // this kernel's share of iterations is spent: the tail kernel continues the
        // same iteration from this state (it, frames, flags), with 16 lanes per face
        // one atomic per wave, on the counter of the wave's own sub-list: every active
        // lane here appends a face
        const int sl = AXIS * NSLOT + (int)wave_slot();
        const unsigned long long mask = __ballot(1);
        const int lane = __lane_id();
        const int leader = __builtin_ctzll(mask);
        int first = 0;
        if (lane == leader) first = atomicAdd(&S.tail_count[sl], __popcll(mask));
        first = __shfl(first, leader, 64);
        const int64_t pos = first + __popcll(mask & ((1ull << lane) - 1ull));
        if (pos < P.tail_cap) { // always true: tail_cap covers every wave of the slot
            const int64_t e = (int64_t)sl * P.tail_cap + pos;
            const int64_t nf = P.tail_n;
            S.tail_f[e] = (int)f;
            S.tail_s[0 * nf + e] = u[0];
            S.tail_s[1 * nf + e] = u[1];
            S.tail_s[2 * nf + e] = T;
            S.tail_s[3 * nf + e] = upp[0];
            S.tail_s[4 * nf + e] = upp[1];
            S.tail_s[5 * nf + e] = Tpp;
            S.tail_meta[e] = it | ((have_pp ? 1 : 0) << 16) | ((restarted ? 1 : 0) << 17);
        }
        // the tail reads the start state of the face's 8 stencil cells: they wait for the
        // update after the tail (the update beside it takes the other cells)
        const double t = S.tstart[0];
#pragma unroll 1
        for (int q = 0; q < 8; ++q) {
            int ci, cj;
            tail_cell<AXIS>(P, f, q, ci, cj);
            const CellRef cr = map2d(P, ci, cj, t);
            if (cr.src >= 0) S.tblock[cr.src] = 1;
        }
        return;
    }
    bool has_frame = true;
    if (failed || !conv) {
        R sm = sqrt(T_m), inv_sm = R(1) / sm;
        R a[10], b[10];
        own_half_2d<R, false, AXIS, REG>(L, NT, idx[0], false, um[0], um[1], inv_sm, a);
        own_half_2d<R, false, AXIS, REG>(L, NT, idx[1], true, um[0], um[1], inv_sm, b);
        for (int k = 0; k < 10; ++k) mf[k] = a[k] + b[k];
        own_half_2d<R, true, AXIS>(L, NT, idx[0], false, um[0], um[1], inv_sm, a);
        own_half_2d<R, true, AXIS>(L, NT, idx[1], true, um[0], um[1], inv_sm, b);
        for (int k = 0; k < 10; ++k) mg[k] = a[k] + b[k];
        R rho = mf[0];
        R dux = sm * mf[1] / rho, duy = sm * mf[2] / rho;
        R Tn = (R(0.5) * sm * sm * (mf[3] + mf[5] - (mf[1] * mf[1] + mf[2] * mf[2]) / rho) + mg[0]) /
               ((R)P.Cv * rho);
        ul[0] = um[0];
        ul[1] = um[1];
        sl = sm;
        if (rho > R(0) && Tn > R(0) && isfinite(Tn) && isfinite(dux) && isfinite(duy)) {
            u[0] = um[0] + dux;
            u[1] = um[1] + duy;
            T = Tn;
        } else {
            has_frame = false;
            u[0] = um[0];
            u[1] = um[1];
            T = T_m;
        }
        cnt.fallback += 1;
    }
    {
        R s = sqrt(T);
        R vx = s * node<R>(3) + fabs(u[0]), vy = s * node<R>(3) + fabs(u[1]);
        if (vx * (R)(0.5 * dt) > (R)(0.5 * P.dx) || vy * (R)(0.5 * dt) > (R)(0.5 * P.dy)) cnt.depout += 1;
    }
    if (!conv) cnt.nonconv += 1;
    cnt.iters += it;
    if ((unsigned long long)it > cnt.itmax) cnt.itmax = it;
    face_write<2, R>(P, S, f, mf, mg, ul, sl, u, T, has_frame, dt);
    S.fiter[f] = it | ((conv ? 0 : 1) << 16) | ((failed ? 1 : 0) << 17);
}

// ---------------------------------------------------------------------------------
// face kernels
// ---------------------------------------------------------------------------------

// 1D: one thread per face. Tubes are laid out in a padded index space with two ghost
// slots on each side: face f of tube k has its stencil at padded slots f + 3k .. f + 3k + 3.
template <typename R, int LIM>
__global__ __launch_bounds__(256) void face_kernel_1d(Params P, State<R> S, int tube_span)
{
    extern __shared__ unsigned char smem_raw[];
    R *L = reinterpret_cast<R *>(smem_raw);
    const int B = blockDim.x;
    const int NT = B + 3 + 3 * tube_span;
    const int64_t f0 = (int64_t)blockIdx.x * B;
    const int64_t f = f0 + threadIdx.x;
    const int64_t flast = min(f0 + B, P.nface) - 1;
    const int k0 = S.face_inst ? S.face_inst[f0] : 0;
    const int k1 = S.face_inst ? S.face_inst[flast] : 0;
    const int64_t vlo = f0 + 3 * (int64_t)k0;
    const int64_t vhi = flast + 3 * (int64_t)k1 + 3;
    // all instances in one block share nothing but the LDS tile; each cell uses its
    // own instance's dt and clock
    for (int64_t v = vlo + threadIdx.x; v <= vhi; v += B) {
        int k = k0;
        while (k < k1 && v >= S.pad_off[k + 1]) ++k;
        const int64_t c0 = S.cell_off[k];
        const int n = (int)(S.cell_off[k + 1] - c0);
        int q = (int)(v - S.pad_off[k]) - 2;
        CellRef c{0, 0, 0, -1, 0};
        if (q >= 0 && q < n) {
            c.src = c0 + q;
        } else {
            int side = (q < 0) ? 0 : 1;
            int sq = side_rule(P, side, q, n, 0.0, xcen(P, q), 0.0, S.tstart[k], c.mx, c.fside, c.falt);
            c.src = (sq < 0) ? -1 : c0 + sq;
        }
        plus_record<1, R>(P, S, c, S.dt[k], L + (v - vlo), NT, 0);
    }
    __syncthreads();
    FaceCount cnt{0, 0, 0, 0, 0, 0, 0};
    unsigned long long nfc = 0;
    if (f < P.nface) {
        const int k = S.face_inst ? S.face_inst[f] : 0;
        const double dt = S.dt[k];
        if (dt > 0.0) {
            const int base = (int)(f + 3 * (int64_t)k - vlo);
            const int idx[4] = {base + 1, base + 2, base, base + 3};
            face_1d<R, LIM>(P, S, L, NT, idx, f, dt, S.dxk ? S.dxk[k] : P.dx, cnt);
            nfc = 1;
        }
    }
    stat_add4(S.stats, ST_FACES, (unsigned)nfc, ST_NONCONV, (unsigned)cnt.nonconv, ST_FALLBACK,
              (unsigned)cnt.fallback, ST_DEPOUT, (unsigned)cnt.depout);
    stat_add32(S.stats, ST_ITERS, (unsigned)cnt.iters);
    stat_max32(S.stats, ST_ITMAX, (unsigned)cnt.itmax);
    if (cnt.depout) atomicOr(S.err, ERR_DEPART);
}

// 2D: thread (i, j) owns x-face (i, j) (if j < ny) and y-face (i, j) (if i < nx).
// LDS tile: cells i0-2 .. i0+BX, j0-2 .. j0+BY.
// NTS: plane stride of the LDS tile (at least (BX+3)(BY+3)), a compile-time constant so
// that the record loads take their plane offsets as immediates; 0: the tile's own size.
// The FP64 Van Leer kernel is held to 2 waves per SIMD: it then spills a few registers,
// and still runs 17% faster than with 1 wave (the FP64 minmod kernel does not gain).
template <typename R, int LIM, int NTS, int REG = 0, int LAY = 0>
__global__ __launch_bounds__(256, (sizeof(R) == 8 && LIM == 0) ? 2 : 1) void face_kernel_2d(Params P, State<R> S)
{
    extern __shared__ unsigned char smem_raw[];
    R *L = reinterpret_cast<R *>(smem_raw);
    const int BX = blockDim.x, BY = blockDim.y;
    const int TX = BX + 3, TY = BY + 3;
    const int NT = NTS ? NTS : TX * TY;
    // the tile of this workgroup: each XCD (own L2) gets a contiguous run of tiles, so that
    // neighbouring tiles, which read the same halo cells, share an L2
    const int tile = xcd_tile((int)(blockIdx.x + gridDim.x * blockIdx.y), (int)(gridDim.x * gridDim.y));
    const int i0 = (tile % (int)gridDim.x) * BX, j0 = (tile / (int)gridDim.x) * BY;
    const double dt = S.dt[0];
    if (!(dt > 0.0)) return;
    const double t = S.tstart[0];
    const int tid = threadIdx.x + BX * threadIdx.y;
    for (int e = tid; e < TX * TY; e += BX * BY) {
        int ci = i0 - 2 + e % TX, cj = j0 - 2 + e / TX;
        // faces reference cells in [-2, nx+1] x [-2, ny+1] only
        if (ci > P.nx + 1 || cj > P.ny + 1) continue;
        CellRef c = map2d(P, ci, cj, t);
        plus_record<2, R, LAY>(P, S, c, dt, L + e, NT, 0);
    }
    __syncthreads();
    const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
    auto li = [&](int ci, int cj) { return (ci - i0 + 2) + TX * (cj - j0 + 2); };
    FaceCount cnt{0, 0, 0, 0, 0, 0, 0};
    unsigned long long nfaces = 0;
    if (i <= P.nx && j < P.ny) {
        const int idx[2] = {li(i - 1, j), li(i, j)};
        face_2d<R, 0, LIM, REG>(P, S, L, NT, idx, 1, TX, (int64_t)i + (int64_t)(P.nx + 1) * j, dt, cnt);
        ++nfaces;
    }
    if (i < P.nx && j <= P.ny) {
        const int idx[2] = {li(i, j - 1), li(i, j)};
        face_2d<R, 1, LIM, REG>(P, S, L, NT, idx, TX, 1, P.nfx + (int64_t)i + (int64_t)P.nx * j, dt, cnt);
        ++nfaces;
    }
    stat_add4(S.stats, ST_FACES, (unsigned)nfaces, ST_NONCONV, (unsigned)cnt.nonconv, ST_FALLBACK,
              (unsigned)cnt.fallback, ST_DEPOUT, (unsigned)cnt.depout);
    stat_add32(S.stats, ST_ITERS, (unsigned)cnt.iters);
    stat_max32(S.stats, ST_ITMAX, (unsigned)cnt.itmax);
    if (cnt.depout) atomicOr(S.err, ERR_DEPART);
}

// ---------------------------------------------------------------------------------
// tail kernel (2D): the faces whose iteration outlasts the face kernel's share
// ---------------------------------------------------------------------------------
//
// A wave of the face kernel runs as long as its slowest face, so the few faces that need
// many iterations would hold 64 lanes each. They continue here with 16 lanes per face: lanes
// 0..7 build the phi-bar-plus records of the 8 stencil cells in LDS; in every iteration lane
// q brings stencil cell q & 7 into the face frame (f for q < 8, g for q >= 8; the order-2
// set of g shifts exactly as the first 6 entries of a degree-3 set), then reconstructs
// population i = q from the 5 cells its upwind direction needs, and the moments are sums
// over the 16 lanes. Same iteration, same stopping rules and finalization as face_2d.

constexpr int TAIL_REC = 8 * Layout<2>::NL; // 8 stencil records
// per stencil cell: f 10, g 6 coefficients (and with REG = 1 the 6 fast f coefficients
// after them), one pad (an odd stride keeps the cells that the lanes of a wave read at one
// time on different LDS banks)
template <int REG>
struct TailDims {
    static constexpr int CSTRIDE = REG ? 23 : 17;
    static constexpr int COEF = 8 * CSTRIDE;
    static constexpr int GROUP = TAIL_REC + COEF;
};

// LDS written by some lanes of a wave and read by others of the same wave
PD void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane permutations inside rows of 16 lanes (DPP): quad_perm [1,0,3,2] and [2,3,0,1]
// (xor 1, xor 2), row_half_mirror (lane i <-> 7 - i in each half-row), row_mirror
// (i <-> 15 - i). Callers run with every lane of the wave active.
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

template <int CTRL>
PD float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
PD double dpp(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// sum over the 16 lanes of a group: quads first, then pairs of quads, then the two
// halves; each stage adds the same two operands in every lane, so all 16 lanes end with
// the same bits
template <typename R>
PD R group_sum(R v)
{
    v += dpp<DPP_XOR1>(v);
    v += dpp<DPP_XOR2>(v);
    v += dpp<DPP_HALF_MIRROR>(v);
    v += dpp<DPP_MIRROR>(v);
    return v;
}

// One face per 16-lane group. Every lane of the wave runs every instruction of the
// iteration (a group that is done, or has no face, computes and discards), so the cross-lane
// sums and the LDS exchange never run under a partial execution mask.
template <typename R, int AXIS, int LIM, int REG = 0, int LAY = 0>
PD void tail_face(const Params &P, const State<R> &S, R *rec, R *coef, int64_t e, bool has,
                  int q, double dt, double t, FaceCount &cnt)
{
    constexpr int CS = TailDims<REG>::CSTRIDE;
    const int64_t nf = P.tail_n;
    const int64_t f = has ? S.tail_f[e] : 0;
    if (has && q < 8) {
        int ci, cj;
        tail_cell<AXIS>(P, f, q, ci, cj);
        CellRef c = map2d(P, ci, cj, t);
        plus_record<2, R, LAY>(P, S, c, dt, rec + q, 8, 0);
    }
    wave_fence();
    const double dn = AXIS ? P.dy : P.dx, dtn = AXIS ? P.dx : P.dy;
    const R hdn = (R)(0.5 * dt / dn), hdt = (R)(0.5 * dt / dtn);
    R u[2] = {R(0), R(0)}, T = R(1), upp[2] = {R(0), R(0)}, Tpp = R(1);
    int it = 0;
    bool have_pp = false, restarted = false;
    if (has) {
        u[0] = S.tail_s[0 * nf + e];
        u[1] = S.tail_s[1 * nf + e];
        T = S.tail_s[2 * nf + e];
        upp[0] = S.tail_s[3 * nf + e];
        upp[1] = S.tail_s[4 * nf + e];
        Tpp = S.tail_s[5 * nf + e];
        const int meta = S.tail_meta[e];
        it = meta & 0xffff;
        have_pp = (meta >> 16) & 1;
        restarted = (meta >> 17) & 1;
    }
    const int it0 = it;
    R um[2] = {R(0), R(0)}, T_m = R(1);
    if (has) mean_frame<2, R>(rec, 8, 0, 1, P, um, T_m);
    // population of this lane: node (cx, cy), Hermite basis values, weight
    const int ix = q & 3, iy = q >> 2;
    const R cx = node<R>(ix), cy = node<R>(iy);
    const R cx2 = cx * cx, cy2 = cy * cy;
    // Hermite basis at the lane's node divided by a! b!, to pair with scaled coefficients
    const R bas[10] = {R(1),
                       cx,
                       cy,
                       R(0.5) * (cx2 - R(1)),
                       cx * cy,
                       R(0.5) * (cy2 - R(1)),
                       cx * (cx2 - R(3)) * R(1.0 / 6.0),
                       R(0.5) * (cx2 - R(1)) * cy,
                       R(0.5) * cx * (cy2 - R(1)),
                       cy * (cy2 - R(3)) * R(1.0 / 6.0)};
    // REG = 1: the basis of the fast coefficients, order 31 22 13 32 23 33
    const R hx2 = R(0.5) * (cx2 - R(1)), hy2 = R(0.5) * (cy2 - R(1));
    const R hx3 = cx * (cx2 - R(3)) * R(1.0 / 6.0), hy3 = cy * (cy2 - R(3)) * R(1.0 / 6.0);
    const R basf[6] = {hx3 * cy, hx2 * hy2, cx * hy3, hx3 * hy2, hx2 * hy3, hx3 * hy3};
    const R wgt = weight1<R>(ix) * weight1<R>(iy);
    const R cn = node<R>(AXIS ? iy : ix), ct = node<R>(AXIS ? ix : iy);
    // stencil cell transformed by this lane
    const int tc = q & 7;
    const bool tg = q >= 8;
    R ul[2] = {u[0], u[1]}, sl = sqrt(T);
    R pf = R(0), pg = R(0);
    bool conv = false, failed = false;
    bool active = has && it < P.max_iter;
    while (__any(active)) {
        if (active) ++it;
        R s, inv_s;
        frame_scale(T, s, inv_s);
        {
            const R r = rec[2 * 8 + tc] * inv_s, dx = (rec[tc] - u[0]) * inv_s,
                    dy = (rec[8 + tc] - u[1]) * inv_s;
            R h[10], mu[10];
            if (!tg) {
                h[0] = rec[3 * 8 + tc];
                h[1] = R(0);
                h[2] = R(0);
#pragma unroll
                for (int k = 0; k < 7; ++k) h[3 + k] = rec[(4 + k) * 8 + tc];
            } else {
#pragma unroll
                for (int k = 0; k < 6; ++k) h[k] = rec[(11 + k) * 8 + tc];
#pragma unroll
                for (int k = 6; k < 10; ++k) h[k] = R(0);
            }
            q2mu_2d(h, mu, 10); // the records hold scaled coefficients
            shift_2d(mu, r, dx, dy, 10);
            mu2q_2d(mu, h, 10);
            R *dst = coef + tc * CS + (tg ? 10 : 0);
            const int nw = tg ? 6 : 10;
#pragma unroll
            for (int k = 0; k < 10; ++k)
                if (k < nw) dst[k] = h[k];
            if (REG && !tg) {
                R hf[6];
                eq_fast_2d(h, hf);
#pragma unroll
                for (int k = 0; k < 6; ++k) dst[16 + k] = hf[k];
            }
        }
        wave_fence();
        const R un = AXIS ? u[1] : u[0], ut = AXIS ? u[0] : u[1];
        const R vn = s * cn + un, vt = s * ct + ut;
        const bool up = vn >= R(0);
        // upwind, downwind, behind-upwind, tangential - and + of the upwind cell
        const int cl[5] = {up ? 0 : 1, up ? 1 : 0, up ? 2 : 3, up ? 4 : 6, up ? 5 : 7};
        R vf[5], vg[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const R *h = coef + cl[m] * CS;
            R a = h[0], b = h[10];
#pragma unroll
            for (int k = 1; k < 10; ++k) a += h[k] * bas[k];
            if (REG) {
#pragma unroll
                for (int k = 0; k < 6; ++k) a += h[16 + k] * basf[k];
            }
#pragma unroll
            for (int k = 1; k < 6; ++k) b += h[10 + k] * bas[k];
            vf[m] = a;
            vg[m] = b;
        }
        wave_fence(); // coefficients are rewritten by the next iteration
        // slopes from limit_part, offsets scaled by limit_scale
        constexpr R sc = R(limit_scale(LIM));
        const R off = (up ? R(0.5) * sc : R(-0.5) * sc) - vn * (hdn * sc), offt = -vt * (hdt * sc);
        auto recon = [&](const R *v) {
            const R A = up ? v[0] - v[2] : v[0] - v[1];
            const R B = up ? v[1] - v[0] : v[2] - v[0];
            const R o = v[0] + off * limit_part(A, B, LIM);
            return o + offt * limit_part(v[0] - v[3], v[4] - v[0], LIM);
        };
        const R pfn = recon(vf), pgn = recon(vg);
        const R wf = wgt * pfn;
        const R rho = group_sum(wf);
        const R m1x = group_sum(wf * cx), m1y = group_sum(wf * cy);
        const R m2 = group_sum(wf * (cx2 + cy2));
        const R g0 = group_sum(wgt * pgn);
        if (active) {
            pf = pfn;
            pg = pgn;
            const R irho = (sizeof(R) == 4) ? frcp(rho) : R(1) / rho;
            const R dux = s * m1x * irho, duy = s * m1y * irho;
            const R rhoe = R(0.5) * s * s * (m2 - (m1x * m1x + m1y * m1y) * irho) + g0;
            const R Tn = temperature(rhoe, rho, irho, P.Cv);
            if (!(rho > R(0)) || !(Tn > R(0)) || !isfinite(Tn) || !isfinite(dux) || !isfinite(duy)) {
                if (!restarted) {
                    restarted = true;
                    u[0] = um[0];
                    u[1] = um[1];
                    T = T_m;
                    have_pp = false;
                } else {
                    failed = true;
                    active = false;
                }
            } else {
                const R unx = u[0] + dux, uny = u[1] + duy;
                const R isq = (sizeof(R) == 4) ? frsq(Tn) : R(1) / sqrt(Tn), iTn = isq * isq;
                const R delta = fmax(fmax(fabs(dux), fabs(duy)) * isq, rel(Tn, T, Tn, iTn));
                const R delta2 =
                    fmax(fmax(fabs(unx - upp[0]), fabs(uny - upp[1])) * isq, rel(Tn, Tpp, Tn, iTn));
                upp[0] = u[0];
                upp[1] = u[1];
                Tpp = T;
                ul[0] = u[0];
                ul[1] = u[1];
                sl = s;
                u[0] = unx;
                u[1] = uny;
                T = Tn;
                if (delta <= (R)P.tol) {
                    conv = true;
                    active = false;
                } else if (have_pp && delta2 <= R(1e-2) * delta) {
                    active = false; // a 2-cycle: stop, not converged
                } else {
                    have_pp = true;
                }
            }
            if (active && it >= P.max_iter) active = false;
        }
    }
    // moments of the last reconstruction (frame ul, sl), degree <= 3 (f) and <= 2 (g)
    R mf[10], mg[10];
    {
        const R mono[10] = {R(1), cx, cy, cx2, cx * cy, cy2, cx2 * cx, cx2 * cy, cx * cy2, cy2 * cy};
        const R wf = wgt * pf, wg = wgt * pg;
#pragma unroll
        for (int k = 0; k < 10; ++k) mf[k] = group_sum(wf * mono[k]);
#pragma unroll
        for (int k = 0; k < 6; ++k) mg[k] = group_sum(wg * mono[k]);
#pragma unroll
        for (int k = 6; k < 10; ++k) mg[k] = R(0);
    }
    if (has) {
        bool has_frame = true;
        if (failed || !conv) {
            R sm = sqrt(T_m), inv_sm = R(1) / sm;
            R a[10], b[10];
            own_half_2d<R, false, AXIS, REG>(rec, 8, 0, false, um[0], um[1], inv_sm, a);
            own_half_2d<R, false, AXIS, REG>(rec, 8, 1, true, um[0], um[1], inv_sm, b);
            for (int k = 0; k < 10; ++k) mf[k] = a[k] + b[k];
            own_half_2d<R, true, AXIS>(rec, 8, 0, false, um[0], um[1], inv_sm, a);
            own_half_2d<R, true, AXIS>(rec, 8, 1, true, um[0], um[1], inv_sm, b);
            for (int k = 0; k < 10; ++k) mg[k] = a[k] + b[k];
            R rho = mf[0];
            R dux = sm * mf[1] / rho, duy = sm * mf[2] / rho;
            R Tn = (R(0.5) * sm * sm * (mf[3] + mf[5] - (mf[1] * mf[1] + mf[2] * mf[2]) / rho) + mg[0]) /
                   ((R)P.Cv * rho);
            ul[0] = um[0];
            ul[1] = um[1];
            sl = sm;
            if (rho > R(0) && Tn > R(0) && isfinite(Tn) && isfinite(dux) && isfinite(duy)) {
                u[0] = um[0] + dux;
                u[1] = um[1] + duy;
                T = Tn;
            } else {
                has_frame = false;
                u[0] = um[0];
                u[1] = um[1];
                T = T_m;
            }
            if (q == 0) cnt.fallback += 1;
        }
        if (q == 0) {
            R s = sqrt(T);
            R vx = s * node<R>(3) + fabs(u[0]), vy = s * node<R>(3) + fabs(u[1]);
            if (vx * (R)(0.5 * dt) > (R)(0.5 * P.dx) || vy * (R)(0.5 * dt) > (R)(0.5 * P.dy)) cnt.depout += 1;
            if (!conv) cnt.nonconv += 1;
            cnt.iters += it;
            cnt.tail_faces += 1;
            cnt.tail_iters += it - it0;
            if ((unsigned long long)it > cnt.itmax) cnt.itmax = it;
            face_write<2, R>(P, S, f, mf, mg, ul, sl, u, T, has_frame, dt);
            S.fiter[f] = it | ((conv ? 0 : 1) << 16) | ((failed ? 1 : 0) << 17);
        }
    }
    wave_fence(); // the records are rebuilt for the group's next face
}

// pre[s] = entries in the axis's sub-lists before s (s = 0..NSLOT), by the block's 256
// threads, one sub-list each; wtot: 4 ints of scratch
PD void tail_prefix(const Params &P, const int *tail_count, int axis, int *pre, int *wtot)
{
    static_assert(NSLOT == 256, "one sub-list per thread of a 256-thread block");
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int x = min(tail_count[axis * NSLOT + tid], P.tail_cap);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    for (int v = 0; v < w; ++v) x += wtot[v];
    pre[tid + 1] = x;
    if (tid == 0) pre[0] = 0;
    __syncthreads();
}

// tail list entry of the axis's k-th face (0 <= k < pre[NSLOT]): in the last sub-list s
// with pre[s] <= k (empty sub-lists are skipped)
PD int64_t tail_entry(const Params &P, const int *pre, int axis, int64_t k)
{
    int lo = 0, hi = NSLOT - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= k)
            lo = mid;
        else
            hi = mid - 1;
    }
    return (int64_t)(axis * NSLOT + lo) * P.tail_cap + (k - pre[lo]);
}

// LDS of one tail block
template <typename R, int REG = 0>
struct TailShared {
    R rec[16 * TailDims<REG>::GROUP];
    int pre[NSLOT + 1];
    int wtot[4];
};

// block bx of nbx (256 threads) of the tail work of one axis
template <typename R, int LIM, int REG = 0, int LAY = 0>
PD void tail_block(const Params &P, const State<R> &S, TailShared<R, REG> &sh, int axis, int bx, int nbx)
{
    R *lds = sh.rec;
    const double dt = S.dt[0];
    if (!(dt > 0.0)) return;
    const double t = S.tstart[0];
    const int q = threadIdx.x & 15, grp = threadIdx.x >> 4;
    R *rec = lds + grp * TailDims<REG>::GROUP, *coef = rec + TAIL_REC;
    // The faces of the axis's NSLOT sub-lists, concatenated, are dealt out 16 per block in
    // turn, so that no block works through a long sub-list alone (the hard faces cluster in
    // the sub-lists of the face-kernel waves that cover a shock).
    {
        // blocks past the axis's last face leave before the prefix (every wave finds the
        // same total, so the whole block leaves)
        const int lane = threadIdx.x & 63;
        int x = 0;
        for (int sl = lane; sl < NSLOT; sl += 64) x += min(S.tail_count[axis * NSLOT + sl], P.tail_cap);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        if ((int64_t)bx * 16 >= x) return;
    }
    int *pre = sh.pre;
    tail_prefix(P, S.tail_count, axis, pre, sh.wtot);
    const int total = pre[NSLOT];
    FaceCount cnt{0, 0, 0, 0, 0, 0, 0};
    // wave-uniform loop: a group without a face in this round takes part with has = false
    for (int64_t k0 = (int64_t)bx * 16; __any(k0 + grp < total); k0 += (int64_t)nbx * 16) {
        const int64_t k = k0 + grp;
        const bool has = k < total;
        int64_t e = 0;
        if (has) e = tail_entry(P, pre, axis, k);
        if (axis == 0)
            tail_face<R, 0, LIM, REG, LAY>(P, S, rec, coef, e, has, q, dt, t, cnt);
        else
            tail_face<R, 1, LIM, REG, LAY>(P, S, rec, coef, e, has, q, dt, t, cnt);
    }
    stat_add4(S.stats, ST_TAIL_FACES, (unsigned)cnt.tail_faces, ST_NONCONV, (unsigned)cnt.nonconv,
              ST_FALLBACK, (unsigned)cnt.fallback, ST_DEPOUT, (unsigned)cnt.depout);
    stat_add32(S.stats, ST_ITERS, (unsigned)cnt.iters);
    stat_add32(S.stats, ST_TAIL_ITERS, (unsigned)cnt.tail_iters);
    stat_max32(S.stats, ST_ITMAX, (unsigned)cnt.itmax);
    if (cnt.depout) atomicOr(S.err, ERR_DEPART);
}

template <typename R, int LIM, int REG = 0, int LAY = 0>
__global__ __launch_bounds__(256) void face_tail_kernel_2d(Params P, State<R> S)
{
    __shared__ TailShared<R, REG> sh;
    tail_block<R, LIM, REG, LAY>(P, S, sh, blockIdx.y, blockIdx.x, gridDim.x);
}

// clears n ints (grid-stride)
__global__ void clear_ints_kernel(int *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// clears the tail counters where no dt_kernel runs before a face kernel (the autotuner)
__global__ void tail_reset_kernel(int *count)
{
    for (int c = threadIdx.x; c < 2 * NSLOT; c += blockDim.x) count[c] = 0;
}

// ---------------------------------------------------------------------------------
// cell update (Sec. III.B.2) + reframe of the next step (Sec. III.B.4)
// ---------------------------------------------------------------------------------

// conserved flux through a face along `axis` (lab frame) from the face state: mass sum f v_a,
// momentum sum f v_b v_a, energy sum (|v|^2/2) f v_a + sum g v_a. Computed in the precision
// of the face state and written with explicit fma, so that the two cells of a face get the
// same bits from whichever kernel updates them: the FP64 flux-form update then telescopes
// exactly between neighbours.
template <int D, typename R>
PD void face_flux(const Params &P, const State<R> &S, int64_t f, int axis, double out[4])
{
    const int64_t nf = P.nface;
    if (D == 1) {
        const R u = S.F[f], T = S.F[nf + f];
        R h[4], hg[2];
        for (int k = 0; k < 4; ++k) h[k] = S.F[(2 + k) * nf + f];
        for (int k = 0; k < 2; ++k) hg[k] = S.F[(6 + k) * nf + f];
        const R s = sqrt(T), rho = h[0], s2 = s * s;
        const R m1 = h[1], m2 = fma(R(2), h[2], h[0]), m3 = fma(R(6), h[3], R(3) * h[1]);
        const R uu = u * u;
        out[0] = (double)fma(rho, u, s * m1);
        out[1] = (double)fma(rho, uu, fma(R(2) * s * u, m1, s2 * m2));
        R e = rho * uu * u;
        e = fma(R(3) * s * uu, m1, e);
        e = fma(R(3) * s2 * u, m2, e);
        e = fma(s2 * s, m3, e);
        out[2] = (double)fma(R(0.5), e, fma(hg[0], u, s * hg[1]));
        out[3] = 0.0;
    } else {
        const R u[2] = {S.F[f], S.F[nf + f]};
        const R T = S.F[2 * nf + f];
        R h[10], hg[3];
        for (int k = 0; k < 10; ++k) h[k] = S.F[(3 + k) * nf + f];
        for (int k = 0; k < 3; ++k) hg[k] = S.F[(13 + k) * nf + f];
        const R s = sqrt(T), rho = h[0], s2 = s * s;
        const R m1[2] = {h[1], h[2]};
        const R m2[2][2] = {{fma(R(2), h[3], h[0]), h[4]}, {h[4], fma(R(2), h[5], h[0])}};
        // mu_30 + mu_12 (axis x) or mu_21 + mu_03 (axis y)
        const R m3c = (axis == 0) ? fma(R(6), h[6], R(3) * h[1]) + fma(R(2), h[8], h[1])
                                  : fma(R(2), h[7], h[2]) + fma(R(6), h[9], R(3) * h[2]);
        const int a = axis;
        const R ua = u[a], m1a = m1[a];
        const R uu = fma(u[0], u[0], u[1] * u[1]);
        const R um1 = fma(u[0], m1[0], u[1] * m1[1]);
        const R trm2 = m2[0][0] + m2[1][1];
        const R ugm2 = fma(u[0], m2[0][a], u[1] * m2[1][a]);
        out[0] = (double)fma(rho, ua, s * m1a);
        for (int b = 0; b < 2; ++b)
            out[1 + b] = (double)fma(rho * u[b], ua, fma(s, fma(u[b], m1a, ua * m1[b]), s2 * m2[b][a]));
        R e = rho * uu * ua;
        e = fma(s * uu, m1a, e);
        e = fma(R(2) * s * ua, um1, e);
        e = fma(R(2) * s2, ugm2, e);
        e = fma(s2 * ua, trm2, e);
        e = fma(s2 * s, m3c, e);
        out[3] = (double)fma(R(0.5), e, fma(hg[0], ua, s * hg[1 + a]));
    }
}

template <int D, typename R, int REG = 0, int LAY = 0>
PD void cell_update(const Params &P, const State<R> &S, int64_t c, int k, double dt, int slot,
                    unsigned long long &bits, bool &all_conv);

// update of cell c (taken = false: no cell for this lane), with the wave-level CFL maximum
// and counters; every lane of the wave calls it
template <int D, typename R, int REG = 0, int LAY = 0>
PD void cell_step(const Params &P, const State<R> &S, int64_t c, bool taken, int slot)
{
    const bool active = taken && c < P.ncell;
    const int k = (active && S.cell_inst) ? S.cell_inst[c] : 0;
    const double dt = S.dt[k];
    const bool work = active && dt > 0.0;
    unsigned long long bits = 0ull;
    bool all_conv = false;
    if (work) cell_update<D, R, REG, LAY>(P, S, c, k, dt, slot, bits, all_conv);
    vmax_update<R>(P, S, slot ^ 1, k, work, bits);
    stat_add4(S.stats, ST_CELLS, work ? 1u : 0u, ST_CONV_CELLS, (work && all_conv) ? 1u : 0u, -1, 0u,
              -1, 0u);
}

template <int D, typename R, int REG = 0, int LAY = 0>
__global__ __launch_bounds__(256) void cell_kernel(Params P, State<R> S, int slot)
{
    // contiguous runs of blocks per XCD: the rows above and below, which share y-faces, in
    // the same L2
    const int64_t blk = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    cell_step<D, R, REG, LAY>(P, S, blk * blockDim.x + threadIdx.x, true, slot);
}

// 1D, resident: one block runs every step of a pond_step call for one tube (block b takes
// tube order[b]), so a step costs no kernel launches and the tube's state stays in the
// caches. Tubes are independent (each has its own dt), so the blocks never wait for each
// other. Each step is the standard one: the tube's dt (one wave), its faces in chunks of
// NT (LDS tile of NT + 3 records, as in face_kernel_1d), then its cells in chunks of NT,
// with block barriers between the phases; per face and per cell the arithmetic is that of
// the launched kernels, so the results are the same bits. Every trip count and branch
// around a barrier depends only on the tube (uniform over the block).
template <typename R, int LIM, int NT>
__global__ __launch_bounds__(NT) void tube_resident_kernel_1d(Params P, State<R> S, double t_end, int nsteps,
                                                               int slot0, const int *order)
{
    extern __shared__ unsigned char smem_raw[];
    R *L = reinterpret_cast<R *>(smem_raw);
    constexpr int NTL = NT + 3;
    const int k = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t c0 = S.cell_off[k], c1 = S.cell_off[k + 1];
    const int n = (int)(c1 - c0);
    const int64_t fa = c0 + k, fz = c1 + k; // the tube's faces fa..fz
    const int64_t pk = S.pad_off[k];
    const double dxa = S.dxk ? S.dxk[k] : P.dx;
    for (int s = 0; s < nsteps; ++s) {
        const int slot = slot0 ^ (s & 1);
        if (tid < 64) instance_dt<1, R>(P, S, k, tid, t_end, slot);
        __syncthreads();
        const double dt = S.dt[k];
        if (dt > 0.0) {
            const double tst = S.tstart[k];
            for (int64_t f0 = fa; f0 <= fz; f0 += NT) {
                const int64_t fl = min(f0 + NT - 1, fz);
                const int64_t vlo = f0 + 3 * (int64_t)k, vhi = fl + 3 * (int64_t)k + 3;
                for (int64_t v = vlo + tid; v <= vhi; v += NT) {
                    const int q = (int)(v - pk) - 2;
                    CellRef c{0, 0, 0, -1, 0};
                    if (q >= 0 && q < n) {
                        c.src = c0 + q;
                    } else {
                        const int side = (q < 0) ? 0 : 1;
                        const int sq = side_rule(P, side, q, n, 0.0, xcen(P, q), 0.0, tst, c.mx, c.fside, c.falt);
                        c.src = (sq < 0) ? -1 : c0 + sq;
                    }
                    plus_record<1, R>(P, S, c, dt, L + (v - vlo), NTL, 0);
                }
                __syncthreads();
                const int64_t f = f0 + tid;
                FaceCount cnt{0, 0, 0, 0, 0, 0, 0};
                unsigned long long nfc = 0;
                if (f <= fl) {
                    const int base = (int)(f + 3 * (int64_t)k - vlo);
                    const int idx[4] = {base + 1, base + 2, base, base + 3};
                    face_1d<R, LIM>(P, S, L, NTL, idx, f, dt, dxa, cnt);
                    nfc = 1;
                }
                stat_add4(S.stats, ST_FACES, (unsigned)nfc, ST_NONCONV, (unsigned)cnt.nonconv, ST_FALLBACK,
                          (unsigned)cnt.fallback, ST_DEPOUT, (unsigned)cnt.depout);
                stat_add32(S.stats, ST_ITERS, (unsigned)cnt.iters);
                stat_max32(S.stats, ST_ITMAX, (unsigned)cnt.itmax);
                if (cnt.depout) atomicOr(S.err, ERR_DEPART);
                __syncthreads();
            }
            for (int64_t b = c0; b < c1; b += NT) cell_step<1, R>(P, S, b + tid, b + tid < c1, slot);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// the semi-Lagrangian realization (Sec. III.A), 1D: one thread per cell
// ---------------------------------------------------------------------------------

// interpolating cubic (Catmull-Rom) weights of the 4 collocation points around a point at
// fraction t in [0, 1) between the middle two
template <typename R>
PD void catmull_rom(R t, R w[4])
{
    const R t2 = t * t, t3 = t2 * t;
    w[0] = R(0.5) * (t2 + t2 - t3 - t);
    w[1] = R(0.5) * (R(3) * t3 - R(5) * t2 + R(2));
    w[2] = R(0.5) * (R(4) * t2 - R(3) * t3 + t);
    w[3] = R(0.5) * (t3 - t2);
}

// Cell c (padded slot c + 4 k + 2 of tube k) advects its populations from the departure
// points x - v_i dt, interpolated from the 4 collocation points (cell centres) around each
// with the Catmull-Rom kernel and clipped into the range of the two that enclose it, all
// transformed into the current frame; the frame is iterated as at the faces (seed: the
// cell's own frame; tolerance, 2-cycle and max_iter stops), then the BGK collision of
// Sec. III.A (2 beta = 2 dt / (2 tau + dt)) acts in the frame of the last advection. The
// new state (conserved variables from the moments, coefficients in the new co-moving
// frame) goes to the staging buffers U2/H2: neighbours still read the old one. The LDS
// tile holds the old state of the block's cells and two ghosts at each tube end (records
// at eps = 0, i.e. the carried populations themselves).
template <typename R>
__global__ __launch_bounds__(256) void sl_kernel_1d(Params P, State<R> S, int span, int slot)
{
    extern __shared__ unsigned char smem_raw[];
    R *L = reinterpret_cast<R *>(smem_raw);
    const int B = blockDim.x;
    const int NT = B + 4 + 4 * span;
    const int64_t c0 = (int64_t)blockIdx.x * B;
    const int64_t c = c0 + threadIdx.x;
    const int64_t clast = min(c0 + B, P.ncell) - 1;
    const int k0 = S.cell_inst ? S.cell_inst[c0] : 0;
    const int k1 = S.cell_inst ? S.cell_inst[clast] : 0;
    const int64_t vlo = c0 + 4 * (int64_t)k0, vhi = clast + 4 * (int64_t)k1 + 4;
    for (int64_t v = vlo + threadIdx.x; v <= vhi; v += B) {
        int k = k0;
        while (k < k1 && v >= S.pad_off[k + 1]) ++k;
        const int64_t cb = S.cell_off[k];
        const int n = (int)(S.cell_off[k + 1] - cb);
        const int q = (int)(v - S.pad_off[k]) - 2;
        CellRef cr{0, 0, 0, -1, 0};
        if (q >= 0 && q < n) {
            cr.src = cb + q;
        } else {
            const int side = (q < 0) ? 0 : 1;
            const int sq = side_rule(P, side, q, n, 0.0, xcen(P, q), 0.0, S.tstart[k], cr.mx, cr.fside, cr.falt);
            cr.src = (sq < 0) ? -1 : cb + sq;
        }
        plus_record<1, R>(P, S, cr, 0.0, L + (v - vlo), NT, 0);
    }
    __syncthreads();
    const bool active = c < P.ncell;
    const int k = (active && S.cell_inst) ? S.cell_inst[c] : 0;
    const double dt = active ? S.dt[k] : 0.0;
    const bool work = active && dt > 0.0;
    FaceCount cnt{0, 0, 0, 0, 0, 0, 0};
    unsigned long long bits = 0ull;
    bool conv = false;
    if (work) {
        const double dxc = S.dxk ? S.dxk[k] : P.dx;
        const int base = (int)(c + 4 * (int64_t)k - vlo); // stencil slots base .. base + 4
        R lu = L[base + 2], lT = L[2 * NT + base + 2];
        R pu = R(0), pT = R(1), fu = lu, fT = lT;
        R pa[4] = {R(0), R(0), R(0), R(0)}, ga[4] = {R(0), R(0), R(0), R(0)};
        bool have_pp = false;
        int it;
        for (it = 1; it <= P.max_iter; ++it) {
            R s, inv_s;
            frame_scale(lT, s, inv_s);
            R Pf[5][4], Pg[5][4];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                cell_pops_1d<R, false>(L, NT, base + m, lu, inv_s, Pf[m]);
                cell_pops_1d<R, true>(L, NT, base + m, lu, inv_s, Pg[m]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const R vi = fma(s, node<R>(i), lu);
                const R d = -vi * (R)(dt / dxc); // departure point, in cells
                if (fabs(d) >= R(1)) cnt.depout += 1;
                const int mb = (d < R(0)) ? 0 : 1; // stencil slot of the point before the base cell
                R w[4];
                catmull_rom(d - R(mb - 1), w);
                R vf = R(0), vg = R(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    vf = fma(w[q], Pf[mb + q][i], vf);
                    vg = fma(w[q], Pg[mb + q][i], vg);
                }
                const R f1 = Pf[mb + 1][i], f2 = Pf[mb + 2][i], g1 = Pg[mb + 1][i], g2 = Pg[mb + 2][i];
                pa[i] = fmin(fmax(vf, fmin(f1, f2)), fmax(f1, f2));
                ga[i] = fmin(fmax(vg, fmin(g1, g2)), fmax(g1, g2));
            }
            fu = lu;
            fT = lT;
            R mf[4], mg[4];
            moments_1d(pa, mf, 4);
            moments_1d(ga, mg, 3);
            const R rho = mf[0];
            const R nu = fma(s, mf[1] / rho, lu);
            // rho E in frame (lu, s): sum (v^2/2) f + sum g, v = lu + s c; T = (E/rho - u^2/2)/C_v
            const R e = R(0.5) * (s * s * mf[2] + R(2) * s * lu * mf[1] + lu * lu * mf[0]) + mg[0];
            const R nT = (e / rho - R(0.5) * nu * nu) / (R)P.Cv;
            if (!(rho > R(0)) || !(nT > R(0)) || !isfinite(nT)) break;
            const R ns = sqrt(nT);
            const R delta = fmax(fabs(nu - lu) / ns, fabs(nT - lT) / nT);
            const R delta2 = fmax(fabs(nu - pu) / ns, fabs(nT - pT) / nT);
            pu = lu;
            pT = lT;
            lu = nu;
            lT = nT;
            if (delta <= (R)P.tol) {
                conv = true;
                break;
            }
            if (have_pp && delta2 <= R(1e-2) * delta) break;
            have_pp = true;
        }
        if (it > P.max_iter) it = P.max_iter;
        cnt.iters = (unsigned long long)it;
        cnt.itmax = (unsigned long long)it;
        cnt.nonconv = conv ? 0ull : 1ull;
        // collision in frame (fu, fT): p <- p + 2 beta (p_eq - p), p_eq = rho (f), g_eq (g)
        R sf, inv_sf;
        frame_scale(fT, sf, inv_sf);
        R mf[4], mg[4];
        moments_1d(pa, mf, 4);
        moments_1d(ga, mg, 3);
        const double rho = (double)mf[0];
        const double eps = dt * rho * (double)fT / P.mu;
        const R b2 = (R)(2.0 * eps / (2.0 + eps));
        const R geq = (R)((P.Cv - 0.5) * rho * (double)fT);
        // moments of the equilibria in their own frame: rho (1, 0, 1, 0), g_eq (1, 0, 1)
        mf[1] = mf[1] - b2 * mf[1];
        mf[2] = fma(b2, (R)rho - mf[2], mf[2]);
        mf[3] = mf[3] - b2 * mf[3];
        mg[0] = fma(b2, geq - mg[0], mg[0]);
        mg[1] = mg[1] - b2 * mg[1];
        mg[2] = fma(b2, geq - mg[2], mg[2]);
        // conserved variables of the new state and its coefficients in the new co-moving frame
        const double su = (double)sf, uu = (double)fu;
        double Un[3];
        Un[0] = (double)mf[0];
        Un[1] = uu * Un[0] + su * (double)mf[1];
        Un[2] = 0.5 * (su * su * (double)mf[2] + 2.0 * su * uu * (double)mf[1] + uu * uu * Un[0]) + (double)mg[0];
        const int64_t n = P.ncell;
        const double irn = 1.0 / Un[0];
        const double un = Un[1] * irn;
        const double Tn = (Un[2] * irn - 0.5 * un * un) / P.Cv;
        const bool ok = (Un[0] > 0.0) && (Tn > 0.0) && isfinite(Tn);
        if (!ok) {
            atomicOr(S.err, ERR_NONPHYS);
            atomicOr(S.inst_err + k, 1);
        }
        const double sn = sqrt(fabs(Tn)), isn = 1.0 / sn;
        const R r = (R)(su * isn), dxs = (R)((uu - un) * isn);
        R hh[4];
        shift_1d(mf, r, dxs, 4);
        mf[0] = (R)Un[0];
        mu2h_1d(mf, hh);
        S.H2[c] = hh[2];
        S.H2[n + c] = hh[3];
        shift_1d(mg, r, dxs, 3);
        mg[3] = R(0);
        mu2h_1d(mg, hh);
        S.H2[2 * n + c] = hh[1];
        S.H2[3 * n + c] = hh[2];
        for (int q = 0; q < 3; ++q) S.U2[q * n + c] = Un[q];
        const double rate = ok ? (fabs(un) + sn * CMAX) / dxc : 0.0;
        bits = (unsigned long long)__double_as_longlong(rate);
    } else if (active) {
        // a frozen or finished tube keeps its state
        const int64_t n = P.ncell;
        for (int q = 0; q < 4; ++q) S.H2[q * n + c] = S.H[q * n + c];
        for (int q = 0; q < 3; ++q) S.U2[q * n + c] = S.U[q * n + c];
    }
    vmax_update<R>(P, S, slot ^ 1, k, work, bits);
    stat_add4(S.stats, ST_FACES, work ? 1u : 0u, ST_NONCONV, (unsigned)cnt.nonconv, ST_CELLS, work ? 1u : 0u,
              ST_CONV_CELLS, (work && conv) ? 1u : 0u);
    stat_add32(S.stats, ST_ITERS, (unsigned)cnt.iters);
    stat_add32(S.stats, ST_DEPOUT, (unsigned)cnt.depout);
    stat_max32(S.stats, ST_ITMAX, (unsigned)cnt.itmax);
    if (cnt.depout) atomicOr(S.err, ERR_DEPART);
}


// the staged state becomes the current one (nh coefficient planes, D + 2 conserved)
template <typename R>
__global__ void sl_commit_kernel(Params P, State<R> S, int nh)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    if (c >= n) return;
    for (int q = 0; q < nh; ++q) S.H[q * n + c] = S.H2[q * n + c];
    for (int q = 0; q < P.dim + 2; ++q) S.U[q * n + c] = S.U2[q * n + c];
}

// The tail work (blocks [0, 2 * TAIL_BLOCKS): TAIL_BLOCKS per axis) beside the update of
// the cells outside the stencils of the tail's faces (the other blocks, 256 cells each),
// whose waves fill the issue slots that the tail's dependency chains leave idle. Neither
// reads a cell that the other writes. Each tail block takes 16 faces a round, so 256 blocks
// per axis finish up to 4,096 faces per axis in one round (the double Mach grid hands over
// about 2,000); the blocks without a face leave at once, but each still has to be dispatched
// ahead of the cell blocks (1,024 per axis cost the launch 2.8 us more).
constexpr int TAIL_BLOCKS = NSLOT;
static_assert((2 * TAIL_BLOCKS) % NXCD == 0, "the cell blocks start on XCD 0");

template <typename R, int LIM, int REG = 0, int LAY = 0>
__global__ __launch_bounds__(256) void tail_cell_kernel_2d(Params P, State<R> S, int slot)
{
    __shared__ TailShared<R, REG> sh;
    if ((int)blockIdx.x < 2 * TAIL_BLOCKS) {
        tail_block<R, LIM, REG, LAY>(P, S, sh, (int)blockIdx.x / TAIL_BLOCKS, (int)blockIdx.x % TAIL_BLOCKS,
                                TAIL_BLOCKS);
        return;
    }
    // 2 * TAIL_BLOCKS is a multiple of the XCD count: cell block k runs on XCD k mod 8
    const int64_t blk = xcd_tile((int)blockIdx.x - 2 * TAIL_BLOCKS, (int)gridDim.x - 2 * TAIL_BLOCKS);
    const int64_t c = blk * 256 + threadIdx.x;
    cell_step<2, R, REG, LAY>(P, S, c, c < P.ncell && !S.tblock[c], slot);
}

// After the tail: the cells in the stencils of its faces (marked by the face kernel), one
// thread per cell of the grid; each clears its mark for the next step.
template <typename R, int REG = 0, int LAY = 0>
__global__ __launch_bounds__(256) void cell_marked_kernel_2d(Params P, State<R> S, int slot)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool marked = c < P.ncell && S.tblock[c] != 0;
    if (!__any(marked)) return;
    if (marked) S.tblock[c] = 0;
    cell_step<2, R, REG, LAY>(P, S, c, marked, slot);
}

template <int D, typename R, int REG, int LAY>
PD void cell_update(const Params &P, const State<R> &S, int64_t c, int k, double dt, int slot,
                    unsigned long long &bits_out, bool &all_conv_out)
{
    const int64_t n = P.ncell;
    const int64_t nf = P.nface;
    double rho, ud[2], T;
    prim<D>(S.U, n, c, rho, ud, T, P.Cv);
    const double sT = sqrt(T);
    const R su = (R)sT, inv_su = (R)(1.0 / sT);
    const R ux = (R)ud[0], uy = (R)ud[1];
    const double eps = dt * rho * T / P.mu;
    const double i2e = 1.0 / (2.0 + eps);
    const R A = (R)((2.0 - eps) * i2e), Bc = (R)(2.0 * eps * i2e);
    const double geq = (P.Cv - 0.5 * D) * rho * T;
    double dU[4] = {0.0, 0.0, 0.0, 0.0};
    bool all_conv = true;
    R mfo[10], mgo[10];
    const double dxc = (D == 1 && S.dxk) ? S.dxk[k] : P.dx;
    // The update of Sec. III.B.2 is linear in the populations, and the new state keeps only
    // their moments of degree <= 3 (f) and <= 2 (g) in the cell frame, so it is done on those
    // moments (mu_a = sum_i W_i p_i c_i^a, dimensionless, in the old cell frame):
    //   mu' = A mu(f~) + Bc mu(f_eq) - sum_faces (dt/dx_n) sgn (s mu_{a+e_n}(q) + u_n mu_a(q)),
    // q the face populations in the cell frame. With the Gauss-Hermite nodes (exact to degree
    // 7 per axis) these equal the sums over the Q populations exactly; the degree-4 moments
    // of the degree-3 expansion q follow from E[c^4] = 3, E[c^4 He_2] = 12, E[c^3 He_1] = 3.
    if (D == 1) {
        R h[4] = {(R)rho, R(0), S.H[c], S.H[n + c]};
        R hg[4] = {(R)(geq - T * (double)h[2]), S.H[2 * n + c], S.H[3 * n + c], R(0)};
        h2mu_1d(h, mfo);
        h2mu_1d(hg, mgo);
        for (int q = 0; q < 4; ++q) {
            mfo[q] *= A;
            mgo[q] *= A;
        }
        mfo[0] += Bc * (R)rho;
        mfo[2] += Bc * (R)rho;
        mgo[0] += Bc * (R)geq;
        mgo[2] += Bc * (R)geq;
        const int64_t fl = c + k; // left face of this cell (tube k)
        for (int side = 0; side < 2; ++side) {
            const int64_t f = fl + side;
            const R sgn = side ? R(1) : R(-1);
            R fu = S.F[f], fT = S.F[nf + f];
            R r = sqrt(fT) * inv_su, d = (fu - ux) * inv_su;
            R hf[4] = {S.F[2 * nf + f], S.F[3 * nf + f], S.F[4 * nf + f], S.F[5 * nf + f]};
            R hgf[4] = {S.F[6 * nf + f], S.F[7 * nf + f], S.F[8 * nf + f], R(0)};
            R mu[4], mg[4];
            h2mu_1d(hf, mu);
            shift_1d(mu, r, d, 4);
            // degree-4 moment of the degree-3 expansion: 3 h0 + 12 h2, h2 = (mu_2 - mu_0) / 2
            const R mu4 = R(6) * mu[2] - R(3) * mu[0];
            h2mu_1d(hgf, mg);
            shift_1d(mg, r, d, 3);
            mg[3] = R(3) * mg[1]; // degree-3 moment of the order-2 g expansion: 3 h1
            const R kf = (R)(dt / dxc) * sgn;
            const R ks = kf * su, ku = kf * ux;
            mfo[0] -= ks * mu[1] + ku * mu[0];
            mfo[1] -= ks * mu[2] + ku * mu[1];
            mfo[2] -= ks * mu[3] + ku * mu[2];
            mfo[3] -= ks * mu4 + ku * mu[3];
            mgo[0] -= ks * mg[1] + ku * mg[0];
            mgo[1] -= ks * mg[2] + ku * mg[1];
            mgo[2] -= ks * mg[3] + ku * mg[2];
            double fl3[4];
            face_flux<1, R>(P, S, f, 0, fl3);
            for (int q3 = 0; q3 < 3; ++q3) dU[q3] -= (dt / dxc) * (double)sgn * fl3[q3];
            all_conv = all_conv && !(S.fiter[f] >> 16);
        }
    } else {
        const int i = (int)(c % P.nx), j = (int)(c / P.nx);
        R h[10] = {(R)rho, R(0), R(0)};
        R hg[10];
        if constexpr (LAY == 1) {
            R fh[7], gh[5];
            coef_from_pops_2d(S.H, n, c, fh, gh);
            for (int q = 0; q < 7; ++q) h[3 + q] = fh[q];
            for (int q = 0; q < 5; ++q) hg[1 + q] = gh[q];
        } else {
            for (int q = 0; q < 7; ++q) h[3 + q] = S.H[q * n + c];
            for (int q = 0; q < 5; ++q) hg[1 + q] = S.H[(7 + q) * n + c];
        }
        hg[0] = (R)(geq - T * ((double)h[3] + (double)h[5]));
        h2mu_2d(h, mfo, 10);
        h2mu_2d(hg, mgo, 6);
#pragma unroll
        for (int q = 0; q < 10; ++q) mfo[q] *= A;
#pragma unroll
        for (int q = 0; q < 6; ++q) mgo[q] *= A;
        mfo[0] += Bc * (R)rho;
        mfo[3] += Bc * (R)rho;
        mfo[5] += Bc * (R)rho;
        mgo[0] += Bc * (R)geq;
        mgo[3] += Bc * (R)geq;
        mgo[5] += Bc * (R)geq;
#pragma unroll 1
        for (int side = 0; side < 4; ++side) {
            const int axis = side >> 1;
            const int hi = side & 1;
            const int64_t f = axis == 0 ? (int64_t)(i + hi) + (int64_t)(P.nx + 1) * j
                                        : P.nfx + (int64_t)i + (int64_t)P.nx * (j + hi);
            const R sgn = hi ? R(1) : R(-1);
            R fux = S.F[f], fuy = S.F[nf + f], fT = S.F[2 * nf + f];
            R r = sqrt(fT) * inv_su, dx = (fux - ux) * inv_su, dy = (fuy - uy) * inv_su;
            R hf[10], mu[10], hgf[10], mg[10];
#pragma unroll
            for (int m = 0; m < 10; ++m) hf[m] = S.F[(3 + m) * nf + f];
#pragma unroll
            for (int m = 0; m < 6; ++m) hgf[m] = S.F[(13 + m) * nf + f];
            // raw moments of the face populations in the cell frame
            h2mu_2d(hf, mu, 10);
            shift_2d(mu, r, dx, dy, 10);
            h2mu_2d(hgf, mg, 6);
            shift_2d(mg, r, dx, dy, 6);
            // degree-3 moments of the order-2 g expansion: mu_30 = 3 h10, mu_21 = h01,
            // mu_12 = h10, mu_03 = 3 h01, with h10 = mu_10, h01 = mu_01
            mg[6] = R(3) * mg[1];
            mg[7] = mg[2];
            mg[8] = mg[1];
            mg[9] = R(3) * mg[2];
            const R kf = (R)(dt / (axis ? P.dy : P.dx)) * sgn;
            const R ks = kf * su, ku = kf * (axis ? uy : ux);
            // degree-4 moments of the face populations that the normal flux needs. Grad: those
            // of the degree-3 expansion, from h00 = mu_00, h20 = (mu_20 - mu_00) / 2,
            // h02 = (mu_02 - mu_00) / 2, h11 = mu_11: mu_22 = h00 + 2 h20 + 2 h02,
            // mu_31 = mu_13 = 3 h11. REG = 1: the product-form equilibrium's with the face
            // state's density and velocity in the cell frame (d = mu_10/mu_00, mu_01/mu_00):
            // mu_22 = rho (dx^2 + 1)(dy^2 + 1), mu_31 = rho (dx^3 + 3 dx) dy, mu_13 likewise.
            // Either way mu_40 = 6 mu_20 - 3 mu_00 on the D1Q4 nodes (roots of He4).
            R m22, m31, m13;
            if (REG) {
                const R ir = R(1) / mu[0];
                const R ddx = mu[1] * ir, ddy = mu[2] * ir;
                m22 = mu[0] * fma(ddx, ddx, R(1)) * fma(ddy, ddy, R(1));
                m31 = mu[0] * ddx * fma(ddx, ddx, R(3)) * ddy;
                m13 = mu[0] * ddy * fma(ddy, ddy, R(3)) * ddx;
            } else {
                m22 = mu[3] + mu[5] - mu[0];
                m31 = R(3) * mu[4];
                m13 = m31;
            }
            if (axis == 0) {
                const R m40 = R(6) * mu[3] - R(3) * mu[0];
                // alpha + e_x: 00->10 10->20 01->11 20->30 11->21 02->12 30->40 21->31 12->22 03->13
                mfo[0] -= ks * mu[1] + ku * mu[0];
                mfo[1] -= ks * mu[3] + ku * mu[1];
                mfo[2] -= ks * mu[4] + ku * mu[2];
                mfo[3] -= ks * mu[6] + ku * mu[3];
                mfo[4] -= ks * mu[7] + ku * mu[4];
                mfo[5] -= ks * mu[8] + ku * mu[5];
                mfo[6] -= ks * m40 + ku * mu[6];
                mfo[7] -= ks * m31 + ku * mu[7];
                mfo[8] -= ks * m22 + ku * mu[8];
                mfo[9] -= ks * m13 + ku * mu[9];
                mgo[0] -= ks * mg[1] + ku * mg[0];
                mgo[1] -= ks * mg[3] + ku * mg[1];
                mgo[2] -= ks * mg[4] + ku * mg[2];
                mgo[3] -= ks * mg[6] + ku * mg[3];
                mgo[4] -= ks * mg[7] + ku * mg[4];
                mgo[5] -= ks * mg[8] + ku * mg[5];
            } else {
                const R m04 = R(6) * mu[5] - R(3) * mu[0];
                // alpha + e_y: 00->01 10->11 01->02 20->21 11->12 02->03 30->31 21->22 12->13 03->04
                mfo[0] -= ks * mu[2] + ku * mu[0];
                mfo[1] -= ks * mu[4] + ku * mu[1];
                mfo[2] -= ks * mu[5] + ku * mu[2];
                mfo[3] -= ks * mu[7] + ku * mu[3];
                mfo[4] -= ks * mu[8] + ku * mu[4];
                mfo[5] -= ks * mu[9] + ku * mu[5];
                mfo[6] -= ks * m31 + ku * mu[6];
                mfo[7] -= ks * m22 + ku * mu[7];
                mfo[8] -= ks * m13 + ku * mu[8];
                mfo[9] -= ks * m04 + ku * mu[9];
                mgo[0] -= ks * mg[2] + ku * mg[0];
                mgo[1] -= ks * mg[4] + ku * mg[1];
                mgo[2] -= ks * mg[5] + ku * mg[2];
                mgo[3] -= ks * mg[7] + ku * mg[3];
                mgo[4] -= ks * mg[8] + ku * mg[4];
                mgo[5] -= ks * mg[9] + ku * mg[5];
            }
            double fl4[4];
            face_flux<2, R>(P, S, f, axis, fl4);
            const double kd = (dt / (axis ? P.dy : P.dx)) * (double)sgn;
            for (int q4 = 0; q4 < 4; ++q4) dU[q4] -= kd * fl4[q4];
            all_conv = all_conv && !(S.fiter[f] >> 16);
        }
    }
    // FP64 conserved update (flux form: exact telescoping between neighbours)
    double Un[4];
    for (int q = 0; q < D + 2; ++q) Un[q] = S.U[q * n + c] + dU[q];
    const double rn = Un[0], irn = 1.0 / rn;
    double un[2] = {Un[1] * irn, D == 2 ? Un[2] * irn : 0.0};
    double ke = un[0] * un[0] + un[1] * un[1];
    double Tn = (Un[D + 1] * irn - 0.5 * ke) / P.Cv;
    bool ok = (rn > 0.0) && (Tn > 0.0) && isfinite(Tn) && isfinite(ke);
    if (!ok) {
        atomicOr(S.err, ERR_NONPHYS);
        atomicOr(S.inst_err + k, 1);
    }
    double sn = sqrt(fabs(Tn)), isn = 1.0 / sn;
    // reframe: non-equilibrium coefficients of the updated populations in the new
    // co-moving frame (Sec. II.C with u' = u, T' = T)
    R r = (R)(sT * isn), dxs = (R)((ud[0] - un[0]) * isn), dys = (R)((ud[1] - un[1]) * isn);
    if (D == 1) {
        R hh[4];
        shift_1d(mfo, r, dxs, 4);
        mfo[0] = (R)rn;
        mu2h_1d(mfo, hh);
        S.H[c] = hh[2];
        S.H[n + c] = hh[3];
        shift_1d(mgo, r, dxs, 3);
        mgo[3] = R(0);
        mu2h_1d(mgo, hh);
        S.H[2 * n + c] = hh[1];
        S.H[3 * n + c] = hh[2];
    } else {
        R hh[10];
        shift_2d(mfo, r, dxs, dys, 10);
        mfo[0] = (R)rn;
        mu2h_2d(mfo, hh, 10);
        if constexpr (LAY == 1) {
            R fh[7], gh[5];
            for (int q = 0; q < 7; ++q) fh[q] = hh[3 + q];
            shift_2d(mgo, r, dxs, dys, 6);
            mu2h_2d(mgo, hh, 6);
            for (int q = 0; q < 5; ++q) gh[q] = hh[1 + q];
            const double Tp = fabs(Tn);
            const R b0 = (R)((P.Cv - 1.0) * rn * Tp - Tp * ((double)fh[0] + (double)fh[2]));
            pops_from_coef_2d(S.H, n, c, (R)rn, b0, fh, gh);
        } else {
            for (int q = 0; q < 7; ++q) S.H[q * n + c] = hh[3 + q];
            shift_2d(mgo, r, dxs, dys, 6);
            mu2h_2d(mgo, hh, 6);
            for (int q = 0; q < 5; ++q) S.H[(7 + q) * n + c] = hh[1 + q];
        }
    }
    for (int q = 0; q < D + 2; ++q) S.U[q * n + c] = Un[q];
    // CFL rate of the new frame: max_a (|u_a| + sqrt(T) c_max) / dx_a
    double rate = (fabs(un[0]) + sn * CMAX) / dxc;
    if (D == 2) rate = fmax(rate, (fabs(un[1]) + sn * CMAX) / P.dy);
    if (!ok) rate = 0.0;
    bits_out = (unsigned long long)__double_as_longlong(rate);
    all_conv_out = all_conv;
    (void)slot;
    (void)k;
}

// ---------------------------------------------------------------------------------
// initialization and read-out
// ---------------------------------------------------------------------------------

// conserved variables of the initial equilibrium; non-equilibrium coefficients zero;
// rate of the first step; faces unseeded (T = -1)
template <int D, typename R>
__global__ void init_kernel(Params P, State<R> S, const double *prim4, int nh)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    int k = 0;
    unsigned long long bits = 0ull;
    if (c < n) {
        k = S.cell_inst ? S.cell_inst[c] : 0;
        double rho = prim4[c], ux = prim4[n + c], uy = prim4[2 * n + c], p = prim4[3 * n + c];
        double T = p / rho;
        S.U[c] = rho;
        S.U[n + c] = rho * ux;
        if (D == 2) S.U[2 * n + c] = rho * uy;
        double ke = ux * ux + (D == 2 ? uy * uy : 0.0);
        S.U[(1 + D) * n + c] = P.Cv * rho * T + 0.5 * rho * ke;
        for (int q = 0; q < nh; ++q) S.H[q * n + c] = R(0);
        double rate = (fabs(ux) + sqrt(T) * CMAX) / ((D == 1 && S.dxk) ? S.dxk[k] : P.dx);
        if (D == 2) rate = fmax(rate, (fabs(uy) + sqrt(T) * CMAX) / P.dy);
        bits = (unsigned long long)__double_as_longlong(rate);
    }
    vmax_update<R>(P, S, 0, k, c < n, bits);
    if (c < n && S.tblock) S.tblock[c] = 0;
    if (c < P.nface) {
        // no seed yet (T < 0); the velocity planes are cleared so that a read-out of the face
        // frames is defined before any face step (the semi-Lagrangian scheme has none)
        S.F[c] = R(0);
        if (D == 2) S.F[P.nface + c] = R(0);
        S.F[(D == 1 ? 1 : 2) * P.nface + c] = R(-1);
        S.fiter[c] = 0; // read by the learned seed's selection before the first step
    }
}

// rho, ux, uy, T planes from U
// End-of-call summary of the state for pond_stats: each of SUM_BLOCKS blocks walks a
// strided share of the cells and faces and writes one record of SUM_NV doubles: smallest
// density, smallest temperature, the conserved totals (U times the cell volume; dim + 2
// values, the rest 0), the lowest index of a cell with rho <= 0, T <= 0 or a non-finite
// value, and the lowest index of a face whose last iteration did not converge (indices as
// exact doubles, -1 for none). Reductions inside a block run in a fixed tree order and the
// host combines the records in block order, so the totals are reproducible bit for bit.
constexpr int SUM_BLOCKS = 256;
constexpr int SUM_NV = 8;

template <int D>
__global__ __launch_bounds__(256) void summary_kernel(Params P, const double *U, const int *fiter,
                                                      const double *dxk, const int *cell_inst, double *out)
{
    __shared__ double red[SUM_NV][256];
    const int tid = threadIdx.x;
    const int64_t n = P.ncell, stride = (int64_t)SUM_BLOCKS * 256;
    double rmin = INFINITY, tmin = INFINITY, tot[4] = {0.0, 0.0, 0.0, 0.0};
    double bad = INFINITY, nonc = INFINITY;
    const double vol2 = P.dx * P.dy;
    for (int64_t c = (int64_t)blockIdx.x * 256 + tid; c < n; c += stride) {
        double rho, u[2], T;
        prim<D>(U, n, c, rho, u, T, P.Cv);
        rmin = fmin(rmin, rho);
        tmin = fmin(tmin, T);
        const double vol = D == 2 ? vol2 : (dxk ? dxk[cell_inst[c]] : P.dx);
        for (int q = 0; q < D + 2; ++q) tot[q] += U[q * n + c] * vol;
        if (!(rho > 0.0 && T > 0.0 && isfinite(rho) && isfinite(T)) && bad == INFINITY) bad = (double)c;
    }
    for (int64_t f = (int64_t)blockIdx.x * 256 + tid; f < P.nface; f += stride)
        if (((fiter[f] >> 16) & 1) && nonc == INFINITY) nonc = (double)f;
    red[0][tid] = rmin;
    red[1][tid] = tmin;
    for (int q = 0; q < 4; ++q) red[2 + q][tid] = tot[q];
    red[6][tid] = bad;
    red[7][tid] = nonc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            red[0][tid] = fmin(red[0][tid], red[0][tid + h]);
            red[1][tid] = fmin(red[1][tid], red[1][tid + h]);
            for (int q = 0; q < 4; ++q) red[2 + q][tid] += red[2 + q][tid + h];
            red[6][tid] = fmin(red[6][tid], red[6][tid + h]);
            red[7][tid] = fmin(red[7][tid], red[7][tid + h]);
        }
        __syncthreads();
    }
    if (tid < SUM_NV) out[(size_t)blockIdx.x * SUM_NV + tid] = red[tid][0];
}

template <int D>
__global__ void fields_kernel(int64_t n, const double *U, double Cv, double *out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double rho, u[2], T;
    prim<D>(U, n, c, rho, u, T, Cv);
    out[c] = rho;
    out[n + c] = u[0];
    out[2 * n + c] = u[1];
    out[3 * n + c] = T;
}

// populations f~ = W_i (...) and g~ of every cell in its co-moving frame
template <int D, typename R, int REG = 0>
__global__ void pops_kernel(Params P, State<R> S, double *f, double *g, double *frame)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    if (c >= n) return;
    double rho, u[2], T;
    prim<D>(S.U, n, c, rho, u, T, P.Cv);
    const double geq = (P.Cv - 0.5 * D) * rho * T;
    if (D == 1) {
        double h[4] = {rho, 0.0, (double)S.H[c], (double)S.H[n + c]};
        double hg[4] = {geq - T * h[2], (double)S.H[2 * n + c], (double)S.H[3 * n + c], 0.0};
        double p[4], q[4];
        eval_1d(h, p, 3);
        eval_1d(hg, q, 2);
        for (int i = 0; i < 4; ++i) {
            f[i * n + c] = weight1<double>(i) * p[i];
            g[i * n + c] = weight1<double>(i) * q[i];
        }
        frame[c] = u[0];
        frame[n + c] = T;
    } else {
        double h[10] = {rho, 0.0, 0.0}, hg[10];
        for (int q = 0; q < 7; ++q) h[3 + q] = S.H[q * n + c];
        hg[0] = geq - T * (h[3] + h[5]);
        for (int q = 0; q < 5; ++q) hg[1 + q] = S.H[(7 + q) * n + c];
        for (int q = 6; q < 10; ++q) hg[q] = 0.0;
        double p[16], q2[16];
        if (REG) {
            // the scaled form (Hermite moments h_ab a! b!) and the six fast ones
            const double q[10] = {h[0], h[1], h[2], 2.0 * h[3], h[4], 2.0 * h[5],
                                  6.0 * h[6], 2.0 * h[7], 2.0 * h[8], 6.0 * h[9]};
            double qf[6];
            eq_fast_2d(q, qf);
            eval_q16_2d(q, qf, p);
        } else {
            eval_2d(h, p, 3);
        }
        eval_2d(hg, q2, 2);
        for (int i = 0; i < 16; ++i) {
            double W = weight1<double>(i & 3) * weight1<double>(i >> 2);
            f[i * n + c] = W * p[i];
            g[i * n + c] = W * q2[i];
        }
        frame[c] = u[0];
        frame[n + c] = u[1];
        frame[2 * n + c] = T;
    }
}

// the 2D state between its two layouts (pond_set_state_layout): coefficients H (12 planes)
// to populations Pp (32 planes), and back
template <typename R>
__global__ void coef_to_pops_kernel_2d(Params P, const double *U, const R *H, R *Pp)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    if (c >= n) return;
    double rho, u[2], T;
    prim<2>(U, n, c, rho, u, T, P.Cv);
    R fh[7], gh[5];
    for (int q = 0; q < 7; ++q) fh[q] = H[q * n + c];
    for (int q = 0; q < 5; ++q) gh[q] = H[(7 + q) * n + c];
    const R b0 = (R)((P.Cv - 1.0) * rho * T - T * ((double)fh[0] + (double)fh[2]));
    pops_from_coef_2d(Pp, n, c, (R)rho, b0, fh, gh);
}

template <typename R>
__global__ void pops_to_coef_kernel_2d(Params P, const R *Pp, R *H)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    if (c >= n) return;
    R fh[7], gh[5];
    coef_from_pops_2d(Pp, n, c, fh, gh);
    for (int q = 0; q < 7; ++q) H[q * n + c] = fh[q];
    for (int q = 0; q < 5; ++q) H[(7 + q) * n + c] = gh[q];
}

// lab-frame moments of the face populations (for comparison with a lab-frame reference)
template <int D, typename R>
__global__ void face_moments_kernel(Params P, State<R> S, double *Mf, double *Mg)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nf = P.nface;
    if (f >= nf) return;
    const int nf3 = (D == 1) ? 4 : 15, ng2 = (D == 1) ? 3 : 7;
    double u[2] = {0, 0}, T, h[10], hg[10];
    if (D == 1) {
        u[0] = S.F[f];
        T = S.F[nf + f];
        for (int k = 0; k < 4; ++k) h[k] = S.F[(2 + k) * nf + f];
        for (int k = 0; k < 3; ++k) hg[k] = S.F[(6 + k) * nf + f];
        hg[3] = 0.0;
        double mu[4], mg[4];
        h2mu_1d(h, mu);
        h2mu_1d(hg, mg);
        // lab moments: shift to frame {0, 1}: x = s c + u
        double s = sqrt(T);
        shift_1d(mu, s, u[0], 4);
        shift_1d(mg, s, u[0], 3);
        for (int k = 0; k < 4; ++k) Mf[f * nf3 + k] = mu[k];
        for (int k = 0; k < 3; ++k) Mg[f * ng2 + k] = mg[k];
    } else {
        u[0] = S.F[f];
        u[1] = S.F[nf + f];
        T = S.F[2 * nf + f];
        for (int k = 0; k < 10; ++k) h[k] = S.F[(3 + k) * nf + f];
        for (int k = 0; k < 6; ++k) hg[k] = S.F[(13 + k) * nf + f];
        double mu[10], mg[10];
        h2mu_2d(h, mu, 10);
        h2mu_2d(hg, mg, 6);
        double s = sqrt(T);
        shift_2d(mu, s, u[0], u[1], 10);
        shift_2d(mg, s, u[0], u[1], 6);
        // packed tensors M0, M1[a], M2[a][b], M3[a][b][c] from mu[k][l] (k x-, l y-degree)
        auto m = [&](const double *v, int kx, int ky) {
            int deg = kx + ky;
            int base = deg == 0 ? 0 : deg == 1 ? 1 : deg == 2 ? 3 : 6;
            return v[base + ky];
        };
        double *o = Mf + f * nf3;
        o[0] = m(mu, 0, 0);
        o[1] = m(mu, 1, 0);
        o[2] = m(mu, 0, 1);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) o[3 + 2 * a + b] = m(mu, (a == 0) + (b == 0), (a == 1) + (b == 1));
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int cc = 0; cc < 2; ++cc)
                    o[7 + 4 * a + 2 * b + cc] =
                        m(mu, (a == 0) + (b == 0) + (cc == 0), (a == 1) + (b == 1) + (cc == 1));
        double *og = Mg + f * ng2;
        og[0] = m(mg, 0, 0);
        og[1] = m(mg, 1, 0);
        og[2] = m(mg, 0, 1);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) og[3 + 2 * a + b] = m(mg, (a == 0) + (b == 0), (a == 1) + (b == 1));
    }
}

} // namespace pond
