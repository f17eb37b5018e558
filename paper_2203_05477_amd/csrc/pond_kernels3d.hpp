// pond_kernels3d.hpp -- the finite-volume PonD step in three dimensions (gfx950, wave64).
//
// Lattice D3Q64: the tensor product of three D1Q4 rules (Sec. II.A, Table I), population
// i = ix + 4 iy + 16 iz. Grad projection of Sec. II.C with the moments of degree <= 3 of f
// (20 of them, q = 20) and <= 2 of g (10). As in 1D and 2D every distribution is held as
// scaled Hermite coefficients q_abc = sum_i W_i p_i He_a(c_ix) He_b(c_iy) He_c(c_iz) in its own
// frame {u, T}, and a change of frame is a binomial shift of the raw dimensionless moments
// (frame-relative: no quantity of size u^3 is formed).
//
// Coefficient order: total degree, then the x exponent descending, then y descending:
//   000 | 100 010 001 | 200 110 101 020 011 002 | 300 210 201 120 111 102 030 021 012 003
// (and the 15 of degree 4 after them where the flux needs them).
//
// Per step four launches on one stream:
//   dt_kernel        the shared one (dt = cfl / rate, clipped at t_end)
//   plus_kernel_3d   one thread per cell: the phi-bar-plus record of Sec. III.B.3 (frame,
//                    density, temperature, coefficients) into a scratch array
//   face_kernel_3d   one launch per axis, four lanes per face: lane n takes the 16
//                    populations of normal node n (their normal velocity, hence their
//                    upwind side, is shared), reconstructs them at the departure points and
//                    forms their share of the moments; a DPP sum over the quad closes the
//                    moments, and the four lanes run the frame iteration in lockstep
//   cell_kernel_3d   one thread per cell: the six face states into the cell frame, flux,
//                    co-moving BGK update (Sec. III.B.2), FP64 conserved update, reframe
//                    (Sec. III.B.4) and the CFL rate of the new frame
//
// Boundaries: periodic, outflow (zero gradient) and reflecting (mirror cell, normal velocity
// and every coefficient of odd degree along the normal reversed) on each of the six sides.
#pragma once

#include <type_traits>

#include "pond_kernels.hpp"

namespace pond {

// compile-time loop: f(std::integral_constant<int, i>) for i = B .. E-1, so that every index
// derived from i inside f is a constant expression (tables below are folded, not evaluated)
template <int B, int E, typename F>
PD void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

struct Geo3 {
    int nx, ny, nz;
    double dx[3];
    int bc[6];         // west, east, south, north, bottom, top: BC_PERIODIC / OUTFLOW / REFLECT
    int64_t nfa[3];    // faces per axis
    int64_t foff[3];   // index of each axis's first face
};

// plane counts: cell coefficients, face state, phi-bar-plus record
constexpr int NH3 = 25;  // f q200..q003 (16), g q100..q002 (9)
constexpr int NF3 = 34;  // u (3), T | f q000..q003 (20) | g q000..q002 (10)
constexpr int NR3 = 32;  // u (3), s, rho, T | f q200..q003 (16) | g q000..q002 (10)
constexpr int R3_U = 0, R3_S = 3, R3_RHO = 4, R3_T = 5, R3_F = 6, R3_G = 22;

// index of the coefficient with exponents (a, b, c) (order above)
__host__ __device__ constexpr int idx3(int a, int b, int c)
{
    return (a + b + c) * (a + b + c + 1) * (a + b + c + 2) / 6 + (b + c) * (b + c + 1) / 2 + c;
}

// exponent of axis `ax` in the coefficient at index o (inverse of idx3)
__host__ __device__ constexpr int exp3(int o, int ax)
{
    for (int d = 0; d <= 4; ++d)
        for (int a = d; a >= 0; --a)
            for (int b = d - a; b >= 0; --b)
                if (idx3(a, b, d - a - b) == o) return ax == 0 ? a : ax == 1 ? b : d - a - b;
    return -1;
}

// parity bits of the coefficient at index o (bit a: odd exponent along axis a)
__host__ __device__ constexpr int par3(int o)
{
    return (exp3(o, 0) & 1) | ((exp3(o, 1) & 1) << 1) | ((exp3(o, 2) & 1) << 2);
}

// the index with exponent e along axis AX and p, q along the two other axes (increasing order)
template <int AX>
__host__ __device__ constexpr int idx_ax(int e, int p, int q)
{
    return AX == 0 ? idx3(e, p, q) : AX == 1 ? idx3(p, e, q) : idx3(p, q, e);
}

// ---------------------------------------------------------------------------------
// one-dimensional maps on the columns of a coefficient set, axis by axis. A column holds the
// values v_0..v_L of one axis's exponent with the other two exponents fixed; DEG is the total
// degree of the set (3: 20 values, 2: 10).
// ---------------------------------------------------------------------------------

// scaled Hermite coefficients -> raw moments: x^2 = He_2 + 1, x^3 = He_3 + 3 He_1
template <typename R>
PD void col_q2mu(R v[4], int L)
{
    if (L >= 3) v[3] = fma(R(3), v[1], v[3]);
    if (L >= 2) v[2] = v[2] + v[0];
}

// raw moments -> scaled Hermite coefficients: He_2 = x^2 - 1, He_3 = x^3 - 3 x
template <typename R>
PD void col_mu2q(R v[4], int L)
{
    if (L >= 3) v[3] = fma(R(-3), v[1], v[3]);
    if (L >= 2) v[2] = v[2] - v[0];
}

// moments of (x + d) from moments of x (binomial)
template <typename R>
PD void col_shift(R v[4], int L, R d)
{
    if (L >= 3) v[3] = fma(d, fma(d, fma(d, v[0], R(3) * v[1]), R(3) * v[2]), v[3]);
    if (L >= 2) v[2] = fma(d, fma(d, v[0], R(2) * v[1]), v[2]);
    if (L >= 1) v[1] = fma(d, v[0], v[1]);
}

// apply a column map (KIND 0: q -> mu, 1: mu -> q, 2: shift by d) along axis AX
template <typename R, int DEG, int AX, int KIND>
PD void axis_pass(R *m, R d)
{
    static_for<0, DEG + 1>([&](auto P) {
        static_for<0, DEG + 1 - decltype(P)::value>([&](auto Qi) {
            constexpr int p = decltype(P)::value, q = decltype(Qi)::value, L = DEG - p - q;
            R v[4];
            v[0] = m[idx_ax<AX>(0, p, q)];
            v[1] = (L >= 1) ? m[idx_ax<AX>(L >= 1 ? 1 : 0, p, q)] : R(0);
            v[2] = (L >= 2) ? m[idx_ax<AX>(L >= 2 ? 2 : 0, p, q)] : R(0);
            v[3] = (L >= 3) ? m[idx_ax<AX>(L >= 3 ? 3 : 0, p, q)] : R(0);
            if constexpr (KIND == 0) col_q2mu(v, L);
            if constexpr (KIND == 1) col_mu2q(v, L);
            if constexpr (KIND == 2) col_shift(v, L, d);
            if constexpr (L >= 1) m[idx_ax<AX>(1, p, q)] = v[1];
            if constexpr (L >= 2) m[idx_ax<AX>(2, p, q)] = v[2];
            if constexpr (L >= 3) m[idx_ax<AX>(3, p, q)] = v[3];
        });
    });
}

template <typename R, int DEG>
PD void q2mu3(R *m)
{
    axis_pass<R, DEG, 0, 0>(m, R(0));
    axis_pass<R, DEG, 1, 0>(m, R(0));
    axis_pass<R, DEG, 2, 0>(m, R(0));
}

template <typename R, int DEG>
PD void mu2q3(R *m)
{
    axis_pass<R, DEG, 0, 1>(m, R(0));
    axis_pass<R, DEG, 1, 1>(m, R(0));
    axis_pass<R, DEG, 2, 1>(m, R(0));
}

// moments of (r c + d) from the raw moments of c, degree <= DEG
template <typename R, int DEG>
PD void shift3(R *m, R r, R dx, R dy, R dz)
{
    const R r2 = r * r, r3 = r2 * r;
    static_for<1, (DEG == 3 ? 20 : 10)>([&](auto O) {
        constexpr int o = decltype(O)::value;
        constexpr int d = exp3(o, 0) + exp3(o, 1) + exp3(o, 2);
        m[o] *= (d == 1) ? r : (d == 2) ? r2 : r3;
    });
    axis_pass<R, DEG, 0, 2>(m, dx);
    axis_pass<R, DEG, 1, 2>(m, dy);
    axis_pass<R, DEG, 2, 2>(m, dz);
}

// raw moment of exponents (a, b, c) of the expansion with scaled coefficients q of degree
// <= KMAX: the product over axes of E[x^m He_k] / k! = m! / (j! 2^j k!), m - k = 2j
__host__ __device__ constexpr double hfac(int m, int k)
{
    if (k > m || ((m - k) & 1)) return 0.0;
    const int j = (m - k) / 2;
    double r = 1.0;
    for (int i = 2; i <= m; ++i) r *= i;
    for (int i = 2; i <= j; ++i) r /= i;
    for (int i = 0; i < j; ++i) r /= 2.0;
    for (int i = 2; i <= k; ++i) r /= i;
    return r;
}

template <typename R, int KMAX, int A, int B, int C>
PD R moment_of_q(const R *q)
{
    R s = R(0);
    static_for<0, 4>([&](auto K0) {
        static_for<0, 4>([&](auto K1) {
            static_for<0, 4>([&](auto K2) {
                constexpr int k0 = decltype(K0)::value, k1 = decltype(K1)::value, k2 = decltype(K2)::value;
                constexpr double w = hfac(A, k0) * hfac(B, k1) * hfac(C, k2);
                if constexpr (k0 + k1 + k2 <= KMAX && w != 0.0) s = fma(R(w), q[idx3(k0, k1, k2)], s);
            });
        });
    });
    return s;
}

// ---------------------------------------------------------------------------------
// populations of one normal node column
// ---------------------------------------------------------------------------------

// 2D index of tangential exponents (b, c) in the order of eval_q_2d: 00 10 01 20 11 02 ...
__host__ __device__ constexpr int idx2(int b, int c) { return (b + c) * (b + c + 1) / 2 + c; }

template <int AXIS>
struct Tan {
    static constexpr int t1 = AXIS == 0 ? 1 : 0;
    static constexpr int t2 = AXIS == 2 ? 1 : 2;
};

// He_a(c_n)/a! at node n, a = 0..3
template <typename R>
PD void node_hermite(int n, R h[4])
{
    const bool inner = (n == 1 || n == 2);
    const R c = node<R>(n);
    h[0] = R(1);
    h[1] = c;
    h[2] = inner ? LatQ<R>::e2a : LatQ<R>::e2b;
    const R e3 = inner ? LatQ<R>::e3a : LatQ<R>::e3b;
    h[3] = (n < 2) ? -e3 : e3;
}

// reduced populations p[t1 + 4 t2] of normal node n (He values hn) from the coefficients q
// (degree DEG): the normal stage A_bc = sum_a q_abc He_a(c_n)/a!, then the tangential
// evaluation of the 2D set A
template <typename R, int DEG, int AXIS>
PD void eval_col3(const R *q, const R hn[4], R p[16])
{
    R A[10];
    static_for<0, DEG + 1>([&](auto Bi) {
        static_for<0, DEG + 1 - decltype(Bi)::value>([&](auto Ci) {
            constexpr int b = decltype(Bi)::value, c = decltype(Ci)::value;
            R s = q[idx_ax<AXIS>(0, b, c)];
            static_for<1, DEG + 1 - b - c>([&](auto Ai) {
                constexpr int a = decltype(Ai)::value;
                s = fma(hn[a], q[idx_ax<AXIS>(a, b, c)], s);
            });
            A[idx2(b, c)] = s;
        });
    });
    eval_q_2d(A, p, DEG);
}

// ---------------------------------------------------------------------------------
// boundaries and the phi-bar-plus records
// ---------------------------------------------------------------------------------

// source cell of (possibly ghost) cell (i, j, k) and its mirror bits (bit a: reflected
// across a side normal to axis a). Stencils reach two cells past a side, and every axis
// has at least two cells.
PD int map3(const Geo3 &G, int i, int j, int k, int &mir)
{
    int c[3] = {i, j, k};
    const int n[3] = {G.nx, G.ny, G.nz};
    mir = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int g = c[a];
        if (g >= 0 && g < n[a]) continue;
        const int kind = G.bc[2 * a + (g < 0 ? 0 : 1)];
        if (kind == BC_PERIODIC) {
            c[a] = (g < 0) ? g + n[a] : g - n[a];
        } else if (kind == BC_REFLECT) {
            c[a] = (g < 0) ? -1 - g : 2 * n[a] - 1 - g;
            mir |= 1 << a;
        } else { // outflow
            c[a] = (g < 0) ? 0 : n[a] - 1;
        }
    }
    return c[0] + G.nx * (c[1] + G.ny * c[2]);
}

// rho, u, T of cell c from the conserved variables
PD void prim3(const double *U, int64_t n, int64_t c, double Cv, double &rho, double u[3], double &T)
{
    rho = U[c];
    const double ir = 1.0 / rho;
    double ke = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = U[(1 + a) * n + c] * ir;
        ke += u[a] * u[a];
    }
    T = (U[4 * n + c] * ir - 0.5 * ke) / Cv;
}

// phi-bar-plus of every cell (Sec. III.B.3): phi+ = A f~ + B f_eq, A = (2 - eps/2)/(2 + eps),
// B = (3 eps/2)/(2 + eps), eps = dt p / mu; f_eq = rho W_i, g_eq = (C_v - 3/2) rho T W_i in
// the co-moving frame (Sec. II.B). g~'s zeroth coefficient follows from the energy:
// rho E = rho |u|^2 / 2 + (T/2)(3 rho + q200 + q020 + q002) + g_0.
template <typename R>
__global__ __launch_bounds__(256) void plus_kernel_3d(Params P, State<R> S, R *rec)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = P.ncell;
    const double dt = S.dt[0];
    if (c >= n || !(dt > 0.0)) return;
    double rho, u[3], T;
    prim3(S.U, n, c, P.Cv, rho, u, T);
    const double eps = dt * rho * T / P.mu;
    const double i2e = 1.0 / (2.0 + eps);
    const double Ap = (2.0 - 0.5 * eps) * i2e, Bp = 1.5 * eps * i2e;
    const double geq = (P.Cv - 1.5) * rho * T;
    const double tr = (double)S.H[0 * n + c] + (double)S.H[3 * n + c] + (double)S.H[5 * n + c];
    const double b0 = geq - 0.5 * T * tr;
#pragma unroll
    for (int a = 0; a < 3; ++a) rec[(R3_U + a) * n + c] = (R)u[a];
    rec[R3_S * n + c] = (R)sqrt(T);
    rec[R3_RHO * n + c] = (R)rho;
    rec[R3_T * n + c] = (R)T;
#pragma unroll
    for (int k = 0; k < 16; ++k) rec[(R3_F + k) * n + c] = (R)(Ap * (double)S.H[k * n + c]);
    rec[R3_G * n + c] = (R)(Ap * b0 + Bp * geq);
#pragma unroll
    for (int k = 0; k < 9; ++k) rec[(R3_G + 1 + k) * n + c] = (R)(Ap * (double)S.H[(16 + k) * n + c]);
}

// a stencil cell's record: frame and coefficients (f: degree 3 with q000 = rho and the
// first-degree ones zero; g: degree 2), mirrored per `mir`
template <typename R>
PD void load_frame3(const R *rec, int64_t n, int src, int mir, R u[3], R &s)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R v = rec[(R3_U + a) * n + src];
        u[a] = ((mir >> a) & 1) ? -v : v;
    }
    s = rec[R3_S * n + src];
}

template <typename R, bool G>
PD void load_coef3(const R *rec, int64_t n, int src, int mir, R *q)
{
    if (!G) {
        q[0] = rec[R3_RHO * n + src];
        q[1] = q[2] = q[3] = R(0);
        static_for<4, 20>([&](auto O) {
            constexpr int o = decltype(O)::value, pm = par3(o);
            const R v = rec[(R3_F + o - 4) * n + src];
            q[o] = (__popc(mir & pm) & 1) ? -v : v;
        });
    } else {
        static_for<0, 10>([&](auto O) {
            constexpr int o = decltype(O)::value, pm = par3(o);
            const R v = rec[(R3_G + o) * n + src];
            q[o] = (__popc(mir & pm) & 1) ? -v : v;
        });
    }
}

// the populations of normal node n of a stencil cell in the face frame (u, s): its
// coefficients shifted into the frame, then evaluated on the column
template <typename R, bool G, int AXIS>
PD void col_pops3(const R *rec, int64_t n, int src, int mir, const R u[3], R inv_s, const R hn[4],
                  R p[16])
{
    constexpr int DEG = G ? 2 : 3;
    R cu[3], cs;
    load_frame3(rec, n, src, mir, cu, cs);
    R q[20];
    load_coef3<R, G>(rec, n, src, mir, q);
    q2mu3<R, DEG>(q);
    shift3<R, DEG>(q, cs * inv_s, (cu[0] - u[0]) * inv_s, (cu[1] - u[1]) * inv_s, (cu[2] - u[2]) * inv_s);
    mu2q3<R, DEG>(q);
    eval_col3<R, DEG, AXIS>(q, hn, p);
}

// the moments of the 16 reduced populations of normal node n (weights W_n c_n^a on the
// normal axis): this lane's share of the raw moments, degree <= DEG
template <typename R, int DEG, int AXIS>
PD void col_moments3(const R p[16], int n, R *m)
{
    R M2[10];
    moments_2d(p, M2, DEG == 3 ? 10 : 6);
    const R c = node<R>(n), w = weight1<R>(n);
    const R wp[4] = {w, w * c, w * c * c, w * c * c * c};
    static_for<0, DEG + 1>([&](auto Ai) {
        static_for<0, DEG + 1 - decltype(Ai)::value>([&](auto Bi) {
            static_for<0, DEG + 1 - decltype(Ai)::value - decltype(Bi)::value>([&](auto Ci) {
                constexpr int a = decltype(Ai)::value, b = decltype(Bi)::value, cc = decltype(Ci)::value;
                m[idx_ax<AXIS>(a, b, cc)] = wp[a] * M2[idx2(b, cc)];
            });
        });
    });
}

// sum over the four lanes of a quad (all four active), then lane 0's sum in every lane:
// the lanes' partial sums come from products that the compiler may fuse into the first
// addition differently in different lanes, and the frame iteration branches on the sums, so
// the four lanes must hold the same bits to stay in step
constexpr int DPP_BCAST0 = 0x00; // quad_perm [0,0,0,0]

template <typename R>
PD R quad_sum(R v)
{
    v = v + dpp<DPP_XOR1>(v);
    v = v + dpp<DPP_XOR2>(v);
    return dpp<DPP_BCAST0>(v);
}

// MUSCL reconstruction of normal node n at the departure points (Sec. III.B.3), its share of
// the moments of phi-bar in the face frame. st: the stencil's source cells, mr: their
// mirror bits (3 per cell), in the order L, R, L-n, R+n, L-t1, L+t1, R-t1, R+t1, L-t2, L+t2,
// R-t2, R+t2. hd*: dt / (2 dx) along the normal and the two tangential axes.
template <typename R, bool G, int AXIS>
PD void recon3(const R *rec, int64_t nc, const int st[12], unsigned long long mr, const R u[3], R s,
               R inv_s, int n, R hdn, R hdt1, R hdt2, int lim, R *m)
{
    constexpr int DEG = G ? 2 : 3;
    constexpr int T1 = Tan<AXIS>::t1, T2 = Tan<AXIS>::t2;
    auto mir = [&](int k) { return (int)((mr >> (3 * k)) & 7ull); };
    R hn[4];
    node_hermite<R>(n, hn);
    const R vn = fma(s, node<R>(n), u[AXIS]);
    const bool up = vn >= R(0);
    const int sU = up ? st[0] : st[1], mU = up ? mir(0) : mir(1);
    const int sB = up ? st[2] : st[0], mB = up ? mir(2) : mir(0);
    const int sF = up ? st[1] : st[3], mF = up ? mir(1) : mir(3);
    const R sc = R(limit_scale(lim));
    R PU[16], T[16], A[16], out[16];
    col_pops3<R, G, AXIS>(rec, nc, sU, mU, u, inv_s, hn, PU);
    col_pops3<R, G, AXIS>(rec, nc, sB, mB, u, inv_s, hn, T);
#pragma unroll
    for (int i = 0; i < 16; ++i) A[i] = PU[i] - T[i];
    col_pops3<R, G, AXIS>(rec, nc, sF, mF, u, inv_s, hn, T);
    const R offn = fma(-vn, hdn * sc, up ? R(0.5) * sc : R(-0.5) * sc);
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = fma(offn, limit_part(A[i], T[i] - PU[i], lim), PU[i]);
    // tangential slopes of the upwind cell
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int base = up ? 4 + 4 * t : 6 + 4 * t;
        const int sm = up ? st[4 + 4 * t] : st[6 + 4 * t], mm = mir(base);
        const int sp = up ? st[5 + 4 * t] : st[7 + 4 * t], mp = mir(base + 1);
        col_pops3<R, G, AXIS>(rec, nc, sm, mm, u, inv_s, hn, T);
#pragma unroll
        for (int i = 0; i < 16; ++i) A[i] = PU[i] - T[i];
        col_pops3<R, G, AXIS>(rec, nc, sp, mp, u, inv_s, hn, T);
        const R ut = t ? u[T2] : u[T1];
        const R hdt = (t ? hdt2 : hdt1) * sc;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const R vt = fma(s, node<R>(t ? (i >> 2) : (i & 3)), ut);
            out[i] = fma(-vt * hdt, limit_part(A[i], T[i] - PU[i], lim), out[i]);
        }
    }
    col_moments3<R, DEG, AXIS>(out, n, m);
}

// first-order upwind state in the neighbours' own frames (the fallback): this lane's share
// of the raw moments in the mean frame (um, sm) of the populations of node n that leave
// L (v >= 0) or R (v < 0)
template <typename R, bool G, int AXIS>
PD void own_half3(const R *rec, int64_t nc, int src, int mir, bool right, const R um[3], R inv_sm,
                  int n, R *m)
{
    constexpr int DEG = G ? 2 : 3;
    constexpr int NM = G ? 10 : 20;
    R cu[3], cs;
    load_frame3(rec, nc, src, mir, cu, cs);
    const R v = fma(cs, node<R>(n), cu[AXIS]);
    const bool take = right ? (v < R(0)) : (v >= R(0));
#pragma unroll
    for (int o = 0; o < NM; ++o) m[o] = R(0);
    if (!take) return;
    R q[20], hn[4], p[16];
    load_coef3<R, G>(rec, nc, src, mir, q);
    node_hermite<R>(n, hn);
    eval_col3<R, DEG, AXIS>(q, hn, p);
    col_moments3<R, DEG, AXIS>(p, n, m);
    shift3<R, DEG>(m, cs * inv_sm, (cu[0] - um[0]) * inv_sm, (cu[1] - um[1]) * inv_sm, (cu[2] - um[2]) * inv_sm);
}

// ---------------------------------------------------------------------------------
// the face kernel
// ---------------------------------------------------------------------------------

// frame from the raw moments (mf: f, degree 3; mg: g) in frame (u, s): density, velocity
// change, temperature
template <typename R>
PD void frame_of3(const R *mf, const R *mg, R s, double Cv, R &rho, R du[3], R &Tn)
{
    rho = mf[0];
    const R irho = (sizeof(R) == 4) ? frcp(rho) : R(1) / rho;
    du[0] = s * mf[1] * irho;
    du[1] = s * mf[2] * irho;
    du[2] = s * mf[3] * irho;
    const R m11 = fma(mf[1], mf[1], fma(mf[2], mf[2], mf[3] * mf[3]));
    const R rhoe = fma(R(0.5) * s * s, mf[4] + mf[7] + mf[9] - m11 * irho, mg[0]);
    Tn = temperature(rhoe, rho, irho, Cv);
}

// The stencil rows of a block's faces in LDS. A block takes FPB consecutive faces of one
// row of faces along x (fixed j, k); their 12-cell stencils lie in a few rows of cells along
// x, each within x0 - 2 .. x0 + FPB + 1 (x0 = the block's first face): 5 rows for the x
// faces (the face row and its four neighbours across), 8 for the y and z faces (the two
// cells on each side along the normal, and the L and R rows' neighbours along the other
// tangential axis). Row r lies at (j + RJ[r], k + RK[r]) relative to the faces' (j, k).
// FPB = 64 in FP32; 32 in FP64, whose records take twice the LDS: a block of 128 threads
// then needs 46 KB (x faces) or 74 KB (y, z), so that two blocks fit a compute unit.
template <typename R>
PD __host__ constexpr int fpb3() { return sizeof(R) == 8 ? 32 : 64; }

template <int AXIS>
struct Rows3 {
    static constexpr int n = AXIS == 0 ? 5 : 8;
    static constexpr int rj(int r)
    {
        if (AXIS == 0) return r == 1 ? -1 : r == 2 ? 1 : 0;
        if (AXIS == 1) {
            constexpr int t[8] = {-1, 0, -2, 1, -1, -1, 0, 0};
            return t[r];
        }
        constexpr int t[8] = {0, 0, 0, 0, -1, 1, -1, 1};
        return t[r];
    }
    static constexpr int rk(int r)
    {
        if (AXIS == 0) return r == 3 ? -1 : r == 4 ? 1 : 0;
        if (AXIS == 1) {
            constexpr int t[8] = {0, 0, 0, 0, -1, 1, -1, 1};
            return t[r];
        }
        constexpr int t[8] = {-1, 0, -2, 1, -1, -1, 0, 0};
        return t[r];
    }
    // stencil cell q (L, R, L-n, R+n, L-t1, L+t1, R-t1, R+t1, L-t2, L+t2, R-t2, R+t2):
    // its row and its x offset from the face index i
    static constexpr int row(int q)
    {
        if (AXIS == 0) {
            constexpr int t[12] = {0, 0, 0, 0, 1, 2, 1, 2, 3, 4, 3, 4};
            return t[q];
        }
        constexpr int t[12] = {0, 1, 2, 3, 0, 0, 1, 1, 4, 5, 6, 7};
        return t[q];
    }
    static constexpr int dx(int q)
    {
        if (AXIS == 0) {
            constexpr int t[12] = {-1, 0, -2, 1, -1, -1, 0, 0, -1, -1, 0, 0};
            return t[q];
        }
        constexpr int t[12] = {0, 0, 0, 0, -1, 1, -1, 1, 0, 0, 0, 0};
        return t[q];
    }
};

// faces per row along x, rows of faces, and the launch's block count for axis AXIS
PD __host__ int face3_rowlen(const Geo3 &G, int axis) { return axis == 0 ? G.nx + 1 : G.nx; }
PD __host__ int64_t face3_rows(const Geo3 &G, int axis)
{
    return axis == 0 ? (int64_t)G.ny * G.nz : axis == 1 ? (int64_t)(G.ny + 1) * G.nz : (int64_t)G.ny * (G.nz + 1);
}
PD __host__ int64_t face3_blocks(const Geo3 &G, int axis, int fpb)
{
    return face3_rows(G, axis) * ((face3_rowlen(G, axis) + fpb - 1) / fpb);
}

// Face f of axis AXIS, four lanes (n = lane & 3). The predictor frame is the previous step's
// face frame (or, before the first step, the frame of the mean conserved variables of L and
// R); the corrector iterates to tol, with the restart from the mean frame, the two-cycle stop
// and the first-order fallback of the 2D kernels. Writes the face state of Sec. III.B.3:
// phi = (phi-bar + (eps/4) phi_eq) / (1 + eps/4) in the final frame, eps = dt p_b / mu.
template <typename R, int AXIS, int LIM>
__global__ __launch_bounds__(4 * fpb3<R>(), sizeof(R) == 8 ? 2 : 1) void face_kernel_3d(Params P, Geo3 G, State<R> S,
                                                                                     const R *grec)
{
    constexpr int FPB = fpb3<R>(), ROW3 = FPB + 4, NTH = 4 * FPB;
    constexpr int NROW = Rows3<AXIS>::n, NRW = NROW * ROW3;
    __shared__ R lds[NR3 * NRW];
    const double dt = S.dt[0];
    if (!(dt > 0.0)) return;
    const int len = face3_rowlen(G, AXIS);
    const int nch = (len + FPB - 1) / FPB;
    const int64_t b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int64_t r = b / nch;
    const int x0 = (int)(b % nch) * FPB;
    const int rows_j = AXIS == 1 ? G.ny + 1 : G.ny;
    const int fj = (int)(r % rows_j), fk = (int)(r / rows_j);
    // fill the LDS rows (mirrored cells stored mirrored); slots past x = nx + 1 are never read
    const int64_t ncg = P.ncell;
    for (int e = threadIdx.x; e < NRW; e += NTH) {
        const int row = e / ROW3, x = x0 - 2 + e % ROW3;
        if (x > G.nx + 1) continue;
        int rj = 0, rk = 0;
        static_for<0, NROW>([&](auto Ri) {
            constexpr int ri = decltype(Ri)::value;
            if (row == ri) {
                rj = Rows3<AXIS>::rj(ri);
                rk = Rows3<AXIS>::rk(ri);
            }
        });
        int mir;
        const int src = map3(G, x, fj + rj, fk + rk, mir);
        static_for<0, NR3>([&](auto Pi) {
            constexpr int pl = decltype(Pi)::value;
            // planes 0-2: velocity; 6-21: f coefficients 4..19; 22-31: g coefficients 0..9
            constexpr int pm = pl < 3 ? (1 << pl) : (pl >= R3_F && pl < R3_G) ? par3(pl - R3_F + 4)
                                                 : pl >= R3_G ? par3(pl - R3_G) : 0;
            const R v = grec[pl * ncg + src];
            lds[pl * NRW + e] = (__popc(mir & pm) & 1) ? -v : v;
        });
    }
    __syncthreads();
    const R *rec = lds;
    const int64_t nc = NRW;
    const int fb = threadIdx.x >> 2, n = threadIdx.x & 3;
    const int i = x0 + fb;
    const int64_t nf = P.nface;
    FaceCount cnt{0, 0, 0, 0, 0, 0, 0};
    bool counted = false;
    if (i < len) {
        counted = (n == 0);
        constexpr int T1 = Tan<AXIS>::t1, T2 = Tan<AXIS>::t2;
        const int64_t f = G.foff[AXIS] + (int64_t)i + (int64_t)len * r;
        int st[12];
        const unsigned long long mr = 0ull;
#pragma unroll
        for (int q = 0; q < 12; ++q) st[q] = Rows3<AXIS>::row(q) * ROW3 + (i - x0 + 2) + Rows3<AXIS>::dx(q);
        const R hdn = (R)(0.5 * dt / G.dx[AXIS]), hdt1 = (R)(0.5 * dt / G.dx[T1]),
                hdt2 = (R)(0.5 * dt / G.dx[T2]);
        // mean frame of L and R (restart frame, first seed), as in the 2D kernels
        R um[3], Tm;
        {
            R uL[3], uR[3], sL, sR;
            load_frame3(rec, nc, st[0], 0, uL, sL);
            load_frame3(rec, nc, st[1], 0, uR, sR);
            const R ra = rec[R3_RHO * nc + st[0]], rb = rec[R3_RHO * nc + st[1]];
            const R Sm = ra + rb, iS = (sizeof(R) == 4) ? frcp(Sm) : R(1) / Sm;
            const R wa = ra * iS, wb = rb * iS;
            R du2 = R(0);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                um[a] = wa * uL[a] + wb * uR[a];
                du2 += (uL[a] - uR[a]) * (uL[a] - uR[a]);
            }
            Tm = wa * rec[R3_T * nc + st[0]] + wb * rec[R3_T * nc + st[1]] + wa * wb * du2 * (R)(0.5 / P.Cv);
        }
        R u[3] = {S.F[0 * nf + f], S.F[1 * nf + f], S.F[2 * nf + f]}, T = S.F[3 * nf + f];
        bool restarted = false;
        if (!(T > R(0))) {
            u[0] = um[0];
            u[1] = um[1];
            u[2] = um[2];
            T = Tm;
            restarted = true;
        }
        R mf[20], mg[10], ul[3] = {u[0], u[1], u[2]}, sl = sqrt(T);
        R upp[3] = {u[0], u[1], u[2]}, Tpp = T;
        bool have_pp = false, conv = false, failed = false;
        int it = 0;
        while (it < P.max_iter) {
            ++it;
            R s, inv_s;
            frame_scale(T, s, inv_s);
            recon3<R, false, AXIS>(rec, nc, st, mr, u, s, inv_s, n, hdn, hdt1, hdt2, LIM, mf);
            recon3<R, true, AXIS>(rec, nc, st, mr, u, s, inv_s, n, hdn, hdt1, hdt2, LIM, mg);
#pragma unroll
            for (int o = 0; o < 20; ++o) mf[o] = quad_sum(mf[o]);
#pragma unroll
            for (int o = 0; o < 10; ++o) mg[o] = quad_sum(mg[o]);
            R rho, du[3], Tn;
            frame_of3(mf, mg, s, P.Cv, rho, du, Tn);
            if (!(rho > R(0)) || !(Tn > R(0)) || !isfinite(Tn) || !isfinite(du[0]) || !isfinite(du[1]) ||
                !isfinite(du[2])) {
                if (!restarted) {
                    restarted = true;
                    u[0] = um[0];
                    u[1] = um[1];
                    u[2] = um[2];
                    T = Tm;
                    have_pp = false;
                    continue;
                }
                failed = true;
                break;
            }
            const R un[3] = {u[0] + du[0], u[1] + du[1], u[2] + du[2]};
            const R isq = (sizeof(R) == 4) ? frsq(Tn) : R(1) / sqrt(Tn), iTn = isq * isq;
            const R dmax = fmax(fmax(fabs(du[0]), fabs(du[1])), fabs(du[2]));
            const R dmax2 = fmax(fmax(fabs(un[0] - upp[0]), fabs(un[1] - upp[1])), fabs(un[2] - upp[2]));
            const R delta = fmax(dmax * isq, rel(Tn, T, Tn, iTn));
            const R delta2 = fmax(dmax2 * isq, rel(Tn, Tpp, Tn, iTn));
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                upp[a] = u[a];
                ul[a] = u[a];
                u[a] = un[a];
            }
            Tpp = T;
            sl = s;
            T = Tn;
            if (delta <= (R)P.tol) {
                conv = true;
                break;
            }
            if (have_pp && delta2 <= R(1e-2) * delta) break; // two-cycle: stop, not converged
            have_pp = true;
        }
        bool has_frame = true;
        if (failed || !conv) {
            const R sm = sqrt(Tm), inv_sm = R(1) / sm;
            R a[20];
            own_half3<R, false, AXIS>(rec, nc, st[0], (int)(mr & 7ull), false, um, inv_sm, n, mf);
            own_half3<R, false, AXIS>(rec, nc, st[1], (int)((mr >> 3) & 7ull), true, um, inv_sm, n, a);
#pragma unroll
            for (int o = 0; o < 20; ++o) mf[o] = quad_sum(mf[o] + a[o]);
            own_half3<R, true, AXIS>(rec, nc, st[0], (int)(mr & 7ull), false, um, inv_sm, n, mg);
            own_half3<R, true, AXIS>(rec, nc, st[1], (int)((mr >> 3) & 7ull), true, um, inv_sm, n, a);
#pragma unroll
            for (int o = 0; o < 10; ++o) mg[o] = quad_sum(mg[o] + a[o]);
            const R rho = mf[0];
            R du[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) du[q] = sm * mf[1 + q] / rho;
            const R m11 = fma(mf[1], mf[1], fma(mf[2], mf[2], mf[3] * mf[3]));
            const R Tn = (R(0.5) * sm * sm * (mf[4] + mf[7] + mf[9] - m11 / rho) + mg[0]) / ((R)P.Cv * rho);
#pragma unroll
            for (int q = 0; q < 3; ++q) ul[q] = um[q];
            sl = sm;
            if (rho > R(0) && Tn > R(0) && isfinite(Tn) && isfinite(du[0]) && isfinite(du[1]) && isfinite(du[2])) {
#pragma unroll
                for (int q = 0; q < 3; ++q) u[q] = um[q] + du[q];
                T = Tn;
            } else {
                has_frame = false;
#pragma unroll
                for (int q = 0; q < 3; ++q) u[q] = um[q];
                T = Tm;
            }
            cnt.fallback += 1;
        }
        {
            const R sT = sqrt(T);
            bool out = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) out = out || (fma(sT, node<R>(3), fabs(u[a])) * (R)(0.5 * dt) > (R)(0.5 * G.dx[a]));
            if (out) cnt.depout += 1;
        }
        if (!conv) cnt.nonconv += 1;
        cnt.iters += it;
        cnt.itmax = it;
        // the face state in the final frame: shift from the frame the moments were taken in
        const R sf = sqrt(T);
        if (has_frame) {
            const R inv = frcp(sf);
            const R r = sl * inv, dx = (ul[0] - u[0]) * inv, dy = (ul[1] - u[1]) * inv, dz = (ul[2] - u[2]) * inv;
            shift3<R, 3>(mf, r, dx, dy, dz);
            shift3<R, 2>(mg, r, dx, dy, dz);
        }
        mu2q3<R, 3>(mf);
        mu2q3<R, 2>(mg);
        const R rho = mf[0];
        R c, e4;
        if constexpr (sizeof(R) == 4) {
            const R eps = has_frame ? (R)(dt / P.mu) * rho * T : R(0);
            e4 = R(0.25) * eps;
            c = frcp(R(1) + e4);
        } else {
            const double eps = has_frame ? dt * (double)rho * (double)T / P.mu : 0.0;
            c = (R)(1.0 / (1.0 + 0.25 * eps));
            e4 = (R)(0.25 * eps);
        }
        // the four lanes hold the same values; each writes every fourth plane
        R outv[NF3];
#pragma unroll
        for (int a = 0; a < 3; ++a) outv[a] = u[a];
        outv[3] = T;
        outv[4] = rho;
#pragma unroll
        for (int o = 1; o < 20; ++o) outv[4 + o] = mf[o] * c;
        outv[24] = (mg[0] + e4 * (R)(P.Cv - 1.5) * rho * T) * c;
#pragma unroll
        for (int o = 1; o < 10; ++o) outv[24 + o] = mg[o] * c;
#pragma unroll
        for (int pl = 0; pl < NF3; ++pl)
            if ((pl & 3) == n) S.F[pl * nf + f] = outv[pl];
        if (n == 0) S.fiter[f] = it | ((conv ? 0 : 1) << 16) | ((failed ? 1 : 0) << 17);
    }
    const unsigned one = counted ? 1u : 0u;
    stat_add4(S.stats, ST_FACES, one, ST_NONCONV, counted ? (unsigned)cnt.nonconv : 0u, ST_FALLBACK,
              counted ? (unsigned)cnt.fallback : 0u, ST_DEPOUT, counted ? (unsigned)cnt.depout : 0u);
    stat_add32(S.stats, ST_ITERS, counted ? (unsigned)cnt.iters : 0u);
    stat_max32(S.stats, ST_ITMAX, counted ? (unsigned)cnt.itmax : 0u);
    if (counted && cnt.depout) atomicOr(S.err, ERR_DEPART);
}

// ---------------------------------------------------------------------------------
// cell update (Sec. III.B.2) and reframe (Sec. III.B.4)
// ---------------------------------------------------------------------------------

// global index of face `side` (2 axis + hi) of cell (i, j, k)
PD int64_t face_of3(const Geo3 &G, int side, int i, int j, int k)
{
    const int axis = side >> 1, hi = side & 1;
    if (axis == 0) return G.foff[0] + (int64_t)(i + hi) + (int64_t)(G.nx + 1) * (j + (int64_t)G.ny * k);
    if (axis == 1) return G.foff[1] + (int64_t)i + (int64_t)G.nx * ((j + hi) + (int64_t)(G.ny + 1) * k);
    return G.foff[2] + (int64_t)i + (int64_t)G.nx * (j + (int64_t)G.ny * (k + hi));
}

// conserved flux through a face along AX from its state (lab frame): mass sum f v_a,
// momentum sum f v_b v_a, energy sum (|v|^2/2) f v_a + sum g v_a, with v = s c + u and the
// raw moments mu (f, degree 3) and mg (g, degree 1) in the face frame. One code path for both
// cells of the face, explicit fma: the FP64 flux-form update telescopes exactly.
template <typename R, int AX>
PD void face_flux3(const R u[3], R s, const R *mu, const R *mg, double out[5])
{
    const R rho = mu[0], s2 = s * s;
    const R m1[3] = {mu[1], mu[2], mu[3]};
    // second moments mu_{e_a + e_b} with b = AX
    const R m2a[3] = {mu[idx3(1 + (AX == 0), AX == 1, AX == 2)], mu[idx3(AX == 0, 1 + (AX == 1), AX == 2)],
                      mu[idx3(AX == 0, AX == 1, 1 + (AX == 2))]};
    // sum_b mu_{2 e_b + e_AX}
    const R m3c = mu[idx3(2 + (AX == 0), AX == 1, AX == 2)] + mu[idx3(AX == 0, 2 + (AX == 1), AX == 2)] +
                  mu[idx3(AX == 0, AX == 1, 2 + (AX == 2))];
    const R ua = u[AX], m1a = m1[AX];
    const R uu = fma(u[0], u[0], fma(u[1], u[1], u[2] * u[2]));
    const R um1 = fma(u[0], m1[0], fma(u[1], m1[1], u[2] * m1[2]));
    const R trm2 = mu[4] + mu[7] + mu[9];
    const R ugm2 = fma(u[0], m2a[0], fma(u[1], m2a[1], u[2] * m2a[2]));
    out[0] = (double)fma(rho, ua, s * m1a);
#pragma unroll
    for (int b = 0; b < 3; ++b)
        out[1 + b] = (double)fma(rho * u[b], ua, fma(s, fma(u[b], m1a, ua * m1[b]), s2 * m2a[b]));
    R e = rho * uu * ua;
    e = fma(s * uu, m1a, e);
    e = fma(R(2) * s * ua, um1, e);
    e = fma(R(2) * s2, ugm2, e);
    e = fma(s2 * ua, trm2, e);
    e = fma(s2 * s, m3c, e);
    out[4] = (double)fma(R(0.5), e, fma(mg[0], ua, s * mg[1 + AX]));
}

// one face of a cell along AX (sgn -1: low side, +1: high side): its conserved flux into dU
// and its populations' contribution to the relaxed moments mfo, mgo (cell frame)
template <typename R, int AX>
PD void side_update3(const Params &P, const Geo3 &G, const State<R> &S, int64_t f, R sgn, double dt,
                     R su, R inv_su, const R uc[3], R *mfo, R *mgo, double dU[5])
{
    const int64_t nf = P.nface;
    const R fu[3] = {S.F[0 * nf + f], S.F[1 * nf + f], S.F[2 * nf + f]};
    const R fT = S.F[3 * nf + f];
    const R fs = sqrt(fT);
    R mu[20], mg[10];
#pragma unroll
    for (int o = 0; o < 20; ++o) mu[o] = S.F[(4 + o) * nf + f];
#pragma unroll
    for (int o = 0; o < 10; ++o) mg[o] = S.F[(24 + o) * nf + f];
    q2mu3<R, 3>(mu);
    q2mu3<R, 2>(mg);
    double fl[5];
    face_flux3<R, AX>(fu, fs, mu, mg, fl);
    const double kd = (dt / G.dx[AX]) * (double)sgn;
#pragma unroll
    for (int q = 0; q < 5; ++q) dU[q] -= kd * fl[q];
    // into the cell frame
    const R r = fs * inv_su;
    const R d3[3] = {(fu[0] - uc[0]) * inv_su, (fu[1] - uc[1]) * inv_su, (fu[2] - uc[2]) * inv_su};
    shift3<R, 3>(mu, r, d3[0], d3[1], d3[2]);
    shift3<R, 2>(mg, r, d3[0], d3[1], d3[2]);
    R qc[20], qg[10];
#pragma unroll
    for (int o = 0; o < 20; ++o) qc[o] = mu[o];
#pragma unroll
    for (int o = 0; o < 10; ++o) qg[o] = mg[o];
    mu2q3<R, 3>(qc);
    mu2q3<R, 2>(qg);
    const R kf = (R)(dt / G.dx[AX]) * sgn;
    const R ks = kf * su, ku = kf * uc[AX];
    static_for<0, 20>([&](auto O) {
        constexpr int o = decltype(O)::value;
        constexpr int a = exp3(o, 0) + (AX == 0), b = exp3(o, 1) + (AX == 1), c = exp3(o, 2) + (AX == 2);
        constexpr int e = idx3(a, b, c);
        R hi;
        if constexpr (e < 20)
            hi = mu[e];
        else
            hi = moment_of_q<R, 3, a, b, c>(qc);
        mfo[o] -= ks * hi + ku * mu[o];
    });
    static_for<0, 10>([&](auto O) {
        constexpr int o = decltype(O)::value;
        constexpr int a = exp3(o, 0) + (AX == 0), b = exp3(o, 1) + (AX == 1), c = exp3(o, 2) + (AX == 2);
        constexpr int e = idx3(a, b, c);
        R hi;
        if constexpr (e < 10)
            hi = mg[e];
        else
            hi = moment_of_q<R, 2, a, b, c>(qg);
        mgo[o] -= ks * hi + ku * mg[o];
    });
}

template <typename R>
PD void cell_update3(const Params &P, const Geo3 &G, const State<R> &S, int64_t c, double dt,
                     unsigned long long &bits_out, bool &all_conv_out)
{
    const int64_t n = P.ncell;
    double rho, ud[3], T;
    prim3(S.U, n, c, P.Cv, rho, ud, T);
    const double sT = sqrt(T);
    const R su = (R)sT, inv_su = (R)(1.0 / sT);
    const R uc[3] = {(R)ud[0], (R)ud[1], (R)ud[2]};
    const double eps = dt * rho * T / P.mu;
    const double i2e = 1.0 / (2.0 + eps);
    const R A = (R)((2.0 - eps) * i2e), Bc = (R)(2.0 * eps * i2e);
    const double geq = (P.Cv - 1.5) * rho * T;
    // moments of f~ and g~ in the cell frame, relaxed: mu' = A mu(f~) + Bc mu(f_eq) (the
    // equilibrium rho W_i has mu_0 = rho, mu_aa = rho, and no other moment up to degree 3)
    R mfo[20], mgo[10];
    mfo[0] = (R)rho;
    mfo[1] = mfo[2] = mfo[3] = R(0);
#pragma unroll
    for (int o = 4; o < 20; ++o) mfo[o] = S.H[(o - 4) * n + c];
    mgo[0] = (R)(geq - 0.5 * T * ((double)mfo[4] + (double)mfo[7] + (double)mfo[9]));
#pragma unroll
    for (int o = 1; o < 10; ++o) mgo[o] = S.H[(15 + o) * n + c];
    q2mu3<R, 3>(mfo);
    q2mu3<R, 2>(mgo);
#pragma unroll
    for (int o = 0; o < 20; ++o) mfo[o] *= A;
#pragma unroll
    for (int o = 0; o < 10; ++o) mgo[o] *= A;
    mfo[0] += Bc * (R)rho;
    mfo[4] += Bc * (R)rho;
    mfo[7] += Bc * (R)rho;
    mfo[9] += Bc * (R)rho;
    mgo[0] += Bc * (R)geq;
    mgo[4] += Bc * (R)geq;
    mgo[7] += Bc * (R)geq;
    mgo[9] += Bc * (R)geq;
    const int i = (int)(c % G.nx);
    const int64_t rr = c / G.nx;
    const int j = (int)(rr % G.ny), k = (int)(rr / G.ny);
    double dU[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    bool all_conv = true;
    // The update is linear in the populations and the new state keeps their moments of
    // degree <= 3 (f) and <= 2 (g) in the cell frame; Gauss-Hermite on the nodes is exact to
    // degree 7 per axis, so with the face populations q in the cell frame
    //   mu' -= (dt/dx_a) sgn (s mu_{e + e_a}(q) + u_a mu_e(q)),
    // and the degree-4 (f) and degree-3 (g) moments are those of the face state's Grad
    // expansion in the cell frame.
#pragma unroll 1
    for (int side = 0; side < 6; ++side) {
        const int64_t f = face_of3(G, side, i, j, k);
        const R sgn = (side & 1) ? R(1) : R(-1);
        switch (side >> 1) {
        case 0: side_update3<R, 0>(P, G, S, f, sgn, dt, su, inv_su, uc, mfo, mgo, dU); break;
        case 1: side_update3<R, 1>(P, G, S, f, sgn, dt, su, inv_su, uc, mfo, mgo, dU); break;
        default: side_update3<R, 2>(P, G, S, f, sgn, dt, su, inv_su, uc, mfo, mgo, dU); break;
        }
        all_conv = all_conv && !(S.fiter[f] >> 16);
    }
    // FP64 conserved update (flux form)
    double Un[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) Un[q] = S.U[q * n + c] + dU[q];
    const double rn = Un[0], irn = 1.0 / rn;
    const double un[3] = {Un[1] * irn, Un[2] * irn, Un[3] * irn};
    const double ke = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
    const double Tn = (Un[4] * irn - 0.5 * ke) / P.Cv;
    const bool ok = (rn > 0.0) && (Tn > 0.0) && isfinite(Tn) && isfinite(ke);
    if (!ok) {
        atomicOr(S.err, ERR_NONPHYS);
        atomicOr(S.inst_err, 1);
    }
    const double sn = sqrt(fabs(Tn)), isn = 1.0 / sn;
    // reframe: coefficients of the updated populations in the new co-moving frame
    const R r = (R)(sT * isn);
    const R d3[3] = {(R)((ud[0] - un[0]) * isn), (R)((ud[1] - un[1]) * isn), (R)((ud[2] - un[2]) * isn)};
    shift3<R, 3>(mfo, r, d3[0], d3[1], d3[2]);
    mfo[0] = (R)rn;
    mu2q3<R, 3>(mfo);
#pragma unroll
    for (int o = 4; o < 20; ++o) S.H[(o - 4) * n + c] = mfo[o];
    shift3<R, 2>(mgo, r, d3[0], d3[1], d3[2]);
    mu2q3<R, 2>(mgo);
#pragma unroll
    for (int o = 1; o < 10; ++o) S.H[(15 + o) * n + c] = mgo[o];
#pragma unroll
    for (int q = 0; q < 5; ++q) S.U[q * n + c] = Un[q];
    double rate = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) rate = fmax(rate, (fabs(un[a]) + sn * CMAX) / G.dx[a]);
    if (!ok) rate = 0.0;
    bits_out = (unsigned long long)__double_as_longlong(rate);
    all_conv_out = all_conv;
}

template <typename R>
__global__ __launch_bounds__(256) void cell_kernel_3d(Params P, Geo3 G, State<R> S, int slot)
{
    const int64_t c = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    const double dt = S.dt[0];
    const bool work = c < P.ncell && dt > 0.0;
    unsigned long long bits = 0ull;
    bool all_conv = false;
    if (work) cell_update3<R>(P, G, S, c, dt, bits, all_conv);
    vmax_update<R>(P, S, slot ^ 1, 0, work, bits);
    stat_add4(S.stats, ST_CELLS, work ? 1u : 0u, ST_CONV_CELLS, (work && all_conv) ? 1u : 0u, -1, 0u, -1, 0u);
}

// ---------------------------------------------------------------------------------
// initialization and read-out
// ---------------------------------------------------------------------------------

// conserved variables of the initial equilibrium (prim5: rho, ux, uy, uz, p planes),
// coefficients zero, rate of the first step, faces unseeded (T = -1)
template <typename R>
__global__ void init_kernel_3d(Params P, Geo3 G, State<R> S, const double *prim5)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    unsigned long long bits = 0ull;
    if (c < n) {
        const double rho = prim5[c], u[3] = {prim5[n + c], prim5[2 * n + c], prim5[3 * n + c]};
        const double T = prim5[4 * n + c] / rho;
        S.U[c] = rho;
        double ke = 0.0, rate = 0.0;
        for (int a = 0; a < 3; ++a) {
            S.U[(1 + a) * n + c] = rho * u[a];
            ke += u[a] * u[a];
            rate = fmax(rate, (fabs(u[a]) + sqrt(T) * CMAX) / G.dx[a]);
        }
        S.U[4 * n + c] = P.Cv * rho * T + 0.5 * rho * ke;
        for (int q = 0; q < NH3; ++q) S.H[q * n + c] = R(0);
        bits = (unsigned long long)__double_as_longlong(rate);
    }
    vmax_update<R>(P, S, 0, 0, c < n, bits);
    if (c < P.nface) {
        for (int a = 0; a < 3; ++a) S.F[a * P.nface + c] = R(0);
        S.F[3 * P.nface + c] = R(-1);
        S.fiter[c] = 0;
    }
}

// end-of-call summary records (as summary_kernel, with five conserved totals):
// rho_min, T_min, totals[5], first bad cell, first non-converged face
constexpr int SUM3_NV = 9;

__global__ __launch_bounds__(256) void summary_kernel_3d(Params P, Geo3 G, const double *U, const int *fiter,
                                                          double *out)
{
    __shared__ double red[SUM3_NV][256];
    const int tid = threadIdx.x;
    const int64_t n = P.ncell, stride = (int64_t)SUM_BLOCKS * 256;
    double rmin = INFINITY, tmin = INFINITY, tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double bad = INFINITY, nonc = INFINITY;
    const double vol = G.dx[0] * G.dx[1] * G.dx[2];
    for (int64_t c = (int64_t)blockIdx.x * 256 + tid; c < n; c += stride) {
        double rho, u[3], T;
        prim3(U, n, c, P.Cv, rho, u, T);
        rmin = fmin(rmin, rho);
        tmin = fmin(tmin, T);
        for (int q = 0; q < 5; ++q) tot[q] += U[q * n + c] * vol;
        if (!(rho > 0.0 && T > 0.0 && isfinite(rho) && isfinite(T)) && bad == INFINITY) bad = (double)c;
    }
    for (int64_t f = (int64_t)blockIdx.x * 256 + tid; f < P.nface; f += stride)
        if (((fiter[f] >> 16) & 1) && nonc == INFINITY) nonc = (double)f;
    red[0][tid] = rmin;
    red[1][tid] = tmin;
    for (int q = 0; q < 5; ++q) red[2 + q][tid] = tot[q];
    red[7][tid] = bad;
    red[8][tid] = nonc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) {
            red[0][tid] = fmin(red[0][tid], red[0][tid + h]);
            red[1][tid] = fmin(red[1][tid], red[1][tid + h]);
            for (int q = 0; q < 5; ++q) red[2 + q][tid] += red[2 + q][tid + h];
            red[7][tid] = fmin(red[7][tid], red[7][tid + h]);
            red[8][tid] = fmin(red[8][tid], red[8][tid + h]);
        }
        __syncthreads();
    }
    if (tid < SUM3_NV) out[(size_t)blockIdx.x * SUM3_NV + tid] = red[tid][0];
}

// rho, ux, uy, T planes (the z velocity is in the conserved variables)
__global__ void fields_kernel_3d(int64_t n, const double *U, double Cv, double *out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double rho, u[3], T;
    prim3(U, n, c, Cv, rho, u, T);
    out[c] = rho;
    out[n + c] = u[0];
    out[2 * n + c] = u[1];
    out[3 * n + c] = T;
}

// populations f~, g~ (64 planes each, i = ix + 4 iy + 16 iz) of every cell in its
// co-moving frame, and the frames (ux, uy, uz, T)
template <typename R>
__global__ void pops_kernel_3d(Params P, State<R> S, double *f, double *g, double *frame)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.ncell;
    if (c >= n) return;
    double rho, u[3], T;
    prim3(S.U, n, c, P.Cv, rho, u, T);
    double q[20], qg[10];
    q[0] = rho;
    q[1] = q[2] = q[3] = 0.0;
    for (int o = 4; o < 20; ++o) q[o] = (double)S.H[(o - 4) * n + c];
    qg[0] = (P.Cv - 1.5) * rho * T - 0.5 * T * (q[4] + q[7] + q[9]);
    for (int o = 1; o < 10; ++o) qg[o] = (double)S.H[(15 + o) * n + c];
    for (int iz = 0; iz < 4; ++iz) {
        double hn[4], p[16], pg[16];
        node_hermite<double>(iz, hn);
        eval_col3<double, 3, 2>(q, hn, p);
        eval_col3<double, 2, 2>(qg, hn, pg);
        for (int t = 0; t < 16; ++t) {
            const double W = weight1<double>(t & 3) * weight1<double>(t >> 2) * weight1<double>(iz);
            f[(t + 16 * iz) * n + c] = W * p[t];
            g[(t + 16 * iz) * n + c] = W * pg[t];
        }
    }
    for (int a = 0; a < 3; ++a) frame[a * n + c] = u[a];
    frame[3 * n + c] = T;
}

// lab-frame moment tensors of the face populations, packed as the oracle packs them:
// f: M0, M1[a], M2[a][b], M3[a][b][c] (40 values); g: M0, M1, M2 (13)
template <typename R>
__global__ void face_moments_kernel_3d(Params P, State<R> S, double *Mf, double *Mg)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nf = P.nface;
    if (f >= nf) return;
    double u[3] = {(double)S.F[f], (double)S.F[nf + f], (double)S.F[2 * nf + f]};
    const double s = sqrt((double)S.F[3 * nf + f]);
    double mu[20], mg[10];
    for (int o = 0; o < 20; ++o) mu[o] = (double)S.F[(4 + o) * nf + f];
    for (int o = 0; o < 10; ++o) mg[o] = (double)S.F[(24 + o) * nf + f];
    q2mu3<double, 3>(mu);
    q2mu3<double, 2>(mg);
    shift3<double, 3>(mu, s, u[0], u[1], u[2]);
    shift3<double, 2>(mg, s, u[0], u[1], u[2]);
    double *o = Mf + f * 40;
    double *og = Mg + f * 13;
    int k = 0;
    auto put = [&](double *dst, const double *src, int deg) {
        int cnt[3];
        for (int w = 0; w < (deg == 0 ? 1 : deg == 1 ? 3 : deg == 2 ? 9 : 27); ++w) {
            cnt[0] = cnt[1] = cnt[2] = 0;
            int x = w;
            for (int d = 0; d < deg; ++d) {
                ++cnt[x % 3];
                x /= 3;
            }
            dst[k++] = src[idx3(cnt[0], cnt[1], cnt[2])];
        }
    };
    for (int deg = 0; deg <= 3; ++deg) put(o, mu, deg);
    k = 0;
    for (int deg = 0; deg <= 2; ++deg) put(og, mg, deg);
}

} // namespace pond
