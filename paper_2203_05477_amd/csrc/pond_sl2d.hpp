// PonD on MI355X (gfx950): the semi-Lagrangian realization of Sec. III.A in two
// dimensions (D2Q16). Included by pond.hip after pond_kernels.hpp, whose helpers it uses
// (records, side rules, the Hermite transforms, statistics); the 1D kernel and the commit
// of the staged state are in pond_kernels.hpp.
#pragma once

namespace pond {

// 2D: one thread per cell, 16 x 16 cells per 256-thread block. The LDS tile holds the
// records (at eps = 0: the carried populations themselves) of the block's cells and two
// layers of neighbours around them, 20 x 20, ghosts through the side rules. Per
// iteration each of the 25 cells of the 5 x 5 stencil around the cell is transformed
// into the current frame once; each population takes the tensor product of the cubic
// kernel along x (the row sums) and along y over the departure point's 4 x 4 centres, and
// is clipped into the range of the 4 centres around its departure point (the cell's own,
// and the neighbours on the departure side along x, along y and diagonally). f first,
// then g: the moments of the advected populations give the next frame. Collision, new
// state and staging as in 1D.
constexpr int SL2_T = 16;             // cells per tile side
constexpr int SL2_W = SL2_T + 4;      // LDS tile side (two neighbours each way)
constexpr int SL2_NT = SL2_W * SL2_W; // records in the tile

// The interpolating cubic as a kernel of the distance x >= 0 to a centre (the Catmull-Rom
// spline, cubic convolution with a = -1/2): 1 - 5/2 x^2 + 3/2 x^3 on [0, 1],
// 2 - 4 x + 5/2 x^2 - 1/2 x^3 on [1, 2], zero beyond. A point at d cells from the middle
// centre (|d| < 1) takes weight K(|d - o|) from the centre at offset o: the 4 around it.
template <typename R>
PD R cubic_kernel(R x)
{
    const R x2 = x * x, x3 = x2 * x;
    const R inner = fma(R(1.5), x3, fma(R(-2.5), x2, R(1)));
    const R outer = fma(R(-0.5), x3, fma(R(2.5), x2, fma(R(-4), x, R(2))));
    return x <= R(1) ? inner : (x < R(2) ? outer : R(0));
}

// advected reduced populations of one kind (f: G = false, g: G = true) in frame (ux, uy,
// s): node column ix departs dx[ix] cells along x, node row iy dy[iy] along y. The row
// sums along x of each stencil row, then the sum along y; the clip range is taken over the
// centres at offsets 0 and -1 (departure on the lower side) or +1 along each axis. One
// stencil cell at a time (loops not unrolled), so that only one cell's populations are
// live. The stencil records come from the block's LDS tile (slot base + a + 20 b for
// stencil cell (a, b)).
template <typename R, bool G, int REG>
PD void sl_advect_2d(const R *L, int base, const float4 *wxl, R ux, R uy, R inv_s, const R dx[4], const R dy[4],
                     R out[16])
{
    R acc[16], lo[16], hi[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        acc[i] = R(0);
        lo[i] = R(INFINITY);
        hi[i] = R(-INFINITY);
    }
#pragma unroll 1
    for (int b = 0; b < 5; ++b) {
        R wy[4];
        bool ry[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wy[k] = cubic_kernel(fabs(dy[k] - R(b - 2)));
            ry[k] = (b == 2) || (b == 1 && dy[k] < R(0)) || (b == 3 && !(dy[k] < R(0)));
        }
        R row[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) row[i] = R(0);
#pragma unroll 1
        for (int a = 0; a < 5; ++a) {
            R wx[4];
            bool cx[4];
            if constexpr (sizeof(R) == 4) {
                // the column's x weights, computed once per iteration (sl_iterate)
                const float4 w4 = wxl[a * 256];
                wx[0] = w4.x;
                wx[1] = w4.y;
                wx[2] = w4.z;
                wx[3] = w4.w;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if constexpr (sizeof(R) != 4) wx[k] = cubic_kernel(fabs(dx[k] - R(a - 2)));
                cx[k] = (a == 2) || (a == 1 && dx[k] < R(0)) || (a == 3 && !(dx[k] < R(0)));
            }
            R p[16];
            cell_pops_2d<R, G, REG>(L, SL2_NT, base + a + SL2_W * b, ux, uy, inv_s, p);
#pragma unroll
            for (int i = 0; i < 16; ++i) row[i] = fma(wx[i & 3], p[i], row[i]);
            // only the 3 x 3 centres around the cell can enclose a departure point (a, b
            // are the same in every lane: a uniform branch)
            if (a >= 1 && a <= 3 && b >= 1 && b <= 3) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const bool in = cx[i & 3] && ry[i >> 2];
                    lo[i] = in ? fmin(lo[i], p[i]) : lo[i];
                    hi[i] = in ? fmax(hi[i], p[i]) : hi[i];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = fma(wy[i >> 2], row[i], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = fmin(fmax(acc[i], lo[i]), hi[i]);
}

// The same advection with the 25 stencil cells on 25 lanes of a 32-lane group (the tail
// kernel): the lane of stencil cell (a, b) (lane = a + 5 b) holds its record `rec`
// (stride 1) and contributes its populations weighted by its kernel weights along x and
// y, and to the clip ranges of the populations whose departure square has its cell at a
// corner; sums, minima and maxima over the group follow (lanes 25..31 add nothing), then
// the group's first lane's results go to every lane, so that all lanes continue on the
// same bits.
template <typename R>
PD R group32_sum(R v)
{
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename R, bool G, int REG>
PD void sl_advect_lanes_2d(const R *rec, bool mine, int a, int b, R ux, R uy, R inv_s, const R dx[4],
                           const R dy[4], R out[16])
{
    R p[16];
    if (mine) {
        cell_pops_2d<R, G, REG>(rec, 1, 0, ux, uy, inv_s, p);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) p[i] = R(0);
    }
    R wx[4], wy[4];
    bool cx[4], ry[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        wx[k] = cubic_kernel(fabs(dx[k] - R(a - 2)));
        wy[k] = cubic_kernel(fabs(dy[k] - R(b - 2)));
        cx[k] = (a == 2) || (a == 1 && dx[k] < R(0)) || (a == 3 && !(dx[k] < R(0)));
        ry[k] = (b == 2) || (b == 1 && dy[k] < R(0)) || (b == 3 && !(dy[k] < R(0)));
    }
    const int lead = (int)(threadIdx.x & ~31u);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const bool in = mine && cx[i & 3] && ry[i >> 2];
        R v = mine ? wy[i >> 2] * (wx[i & 3] * p[i]) : R(0);
        R lo = in ? p[i] : R(INFINITY), hi = in ? p[i] : R(-INFINITY);
        v = group32_sum(v);
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            lo = fmin(lo, __shfl_xor(lo, o, 64));
            hi = fmax(hi, __shfl_xor(hi, o, 64));
        }
        v = __shfl(v, lead, 64);
        out[i] = fmin(fmax(v, lo), hi);
    }
}

// the frame iteration of one cell: the current frame (u, T), the frame one iteration back,
// the iterations done, and the moments of the last advected populations in the frame they
// were taken in (fu, fT)
template <typename R>
struct SlIter {
    R ux, uy, T, pux, puy, pT, fux, fuy, fT;
    int it;
    bool have_pp;
    R mf[10], mg[10];
};

enum { SL_GO = 0, SL_CONVERGED = 1, SL_STOPPED = 2, SL_FAILED = 3 };

// one iteration: advection of f and g from the departure points of the current frame,
// their moments, the next frame, and the stopping rules of the face iteration (tolerance;
// 2-cycle; a non-physical frame ends the cell's iteration)
// LANES: the stencil is spread over a 32-lane group (rec: this lane's record, (a, b) its
// stencil cell, mine: a + 5 b < 25), else it is the block's LDS tile at slot `base`.
template <typename R, int REG, bool LANES>
PD int sl_iterate(const R *L, int base, float4 *wxl, const R *rec, bool mine, int a, int b, R kx, R ky, double Cv,
                  double tol, SlIter<R> &I, unsigned long long &depout)
{
    R s, inv_s;
    frame_scale(I.T, s, inv_s);
    R dxk[4], dyk[4];
    int outx = 0, outy = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        dxk[k] = -fma(s, node<R>(k), I.ux) * kx; // departure point, in cells
        dyk[k] = -fma(s, node<R>(k), I.uy) * ky;
        outx += fabs(dxk[k]) >= R(1);
        outy += fabs(dyk[k]) >= R(1);
    }
    // populations whose departure point leaves the cell's square along either axis
    depout += (unsigned long long)(4 * (outx + outy) - outx * outy);
    if constexpr (!LANES && sizeof(R) == 4) {
        // FP32: the x weights of the 5 stencil columns for the 4 node columns, once per
        // iteration into this thread's LDS slots (read back per stencil cell by both passes)
#pragma unroll
        for (int a = 0; a < 5; ++a)
            wxl[a * 256] = make_float4(cubic_kernel(fabs(dxk[0] - R(a - 2))), cubic_kernel(fabs(dxk[1] - R(a - 2))),
                                       cubic_kernel(fabs(dxk[2] - R(a - 2))), cubic_kernel(fabs(dxk[3] - R(a - 2))));
    }
    {
        R pa[16];
        if constexpr (LANES)
            sl_advect_lanes_2d<R, false, REG>(rec, mine, a, b, I.ux, I.uy, inv_s, dxk, dyk, pa);
        else
            sl_advect_2d<R, false, REG>(L, base, wxl, I.ux, I.uy, inv_s, dxk, dyk, pa);
        moments_2d(pa, I.mf, 10);
    }
    {
        R ga[16];
        if constexpr (LANES)
            sl_advect_lanes_2d<R, true, 0>(rec, mine, a, b, I.ux, I.uy, inv_s, dxk, dyk, ga);
        else
            sl_advect_2d<R, true, 0>(L, base, wxl, I.ux, I.uy, inv_s, dxk, dyk, ga);
        moments_2d(ga, I.mg, 6);
    }
    I.fux = I.ux;
    I.fuy = I.uy;
    I.fT = I.T;
    const R rho = I.mf[0];
    const R nux = fma(s, I.mf[1] / rho, I.ux), nuy = fma(s, I.mf[2] / rho, I.uy);
    // rho E in frame (u, s): sum (|v|^2/2) f + sum g, v = u + s c
    const R e = R(0.5) * (s * s * (I.mf[3] + I.mf[5]) + R(2) * s * (I.ux * I.mf[1] + I.uy * I.mf[2]) +
                          (I.ux * I.ux + I.uy * I.uy) * I.mf[0]) +
                I.mg[0];
    const R nT = (e / rho - R(0.5) * (nux * nux + nuy * nuy)) / (R)Cv;
    if (!(rho > R(0)) || !(nT > R(0)) || !isfinite(nT)) return SL_FAILED;
    const R ns = sqrt(nT);
    const R delta = fmax(fmax(fabs(nux - I.ux), fabs(nuy - I.uy)) / ns, fabs(nT - I.T) / nT);
    const R delta2 = fmax(fmax(fabs(nux - I.pux), fabs(nuy - I.puy)) / ns, fabs(nT - I.pT) / nT);
    I.pux = I.ux;
    I.puy = I.uy;
    I.pT = I.T;
    I.ux = nux;
    I.uy = nuy;
    I.T = nT;
    if (delta <= (R)tol) return SL_CONVERGED;
    if (I.have_pp && delta2 <= R(1e-2) * delta) return SL_STOPPED;
    I.have_pp = true;
    return SL_GO;
}

// the end of a cell's step: the BGK collision in the frame of the last advection
// (p <- p + 2 beta (p_eq - p), 2 beta = 2 eps / (2 + eps), eps = dt p / mu), the
// conserved variables of the new populations and their coefficients in the new co-moving
// frame, into the staging buffers; returns the cell's CFL rate as a bit pattern (0 for a
// non-physical result, which flags the run)
template <typename R>
PD unsigned long long sl_finish(const Params &P, const State<R> &S, int64_t c, double dt, SlIter<R> &I)
{
    R *mf = I.mf, *mg = I.mg;
    R sf, inv_sf;
    frame_scale(I.fT, sf, inv_sf);
    const double rho = (double)mf[0];
    const double eps = dt * rho * (double)I.fT / P.mu;
    const R b2 = (R)(2.0 * eps / (2.0 + eps));
    const R geq = (R)((P.Cv - 1.0) * rho * (double)I.fT);
    // the equilibria's moments in their own frame: rho (f) and g_eq (g) at degrees 00, 20
    // and 02, zero elsewhere
#pragma unroll
    for (int q = 1; q < 10; ++q)
        if (q != 3 && q != 5) mf[q] = mf[q] - b2 * mf[q];
    mf[3] = fma(b2, (R)rho - mf[3], mf[3]);
    mf[5] = fma(b2, (R)rho - mf[5], mf[5]);
    mg[0] = fma(b2, geq - mg[0], mg[0]);
    mg[1] = mg[1] - b2 * mg[1];
    mg[2] = mg[2] - b2 * mg[2];
    mg[3] = fma(b2, geq - mg[3], mg[3]);
    mg[4] = mg[4] - b2 * mg[4];
    mg[5] = fma(b2, geq - mg[5], mg[5]);
    const double su = (double)sf, ux = (double)I.fux, uy = (double)I.fuy;
    double Un[4];
    Un[0] = (double)mf[0];
    Un[1] = ux * Un[0] + su * (double)mf[1];
    Un[2] = uy * Un[0] + su * (double)mf[2];
    Un[3] = 0.5 * (su * su * ((double)mf[3] + (double)mf[5]) + 2.0 * su * (ux * (double)mf[1] + uy * (double)mf[2]) +
                   (ux * ux + uy * uy) * Un[0]) +
            (double)mg[0];
    const int64_t n = P.ncell;
    const double irn = 1.0 / Un[0];
    const double unx = Un[1] * irn, uny = Un[2] * irn;
    const double Tn = (Un[3] * irn - 0.5 * (unx * unx + uny * uny)) / P.Cv;
    const bool ok = (Un[0] > 0.0) && (Tn > 0.0) && isfinite(Tn);
    if (!ok) {
        atomicOr(S.err, ERR_NONPHYS);
        atomicOr(S.inst_err, 1);
    }
    const double sn = sqrt(fabs(Tn)), isn = 1.0 / sn;
    const R r = (R)(su * isn), dxs = (R)((ux - unx) * isn), dys = (R)((uy - uny) * isn);
    R hh[10];
    shift_2d(mf, r, dxs, dys, 10);
    mf[0] = (R)Un[0];
    mu2h_2d(mf, hh, 10);
#pragma unroll
    for (int q = 0; q < 7; ++q) S.H2[q * n + c] = hh[3 + q];
    shift_2d(mg, r, dxs, dys, 6);
    mu2h_2d(mg, hh, 6);
#pragma unroll
    for (int q = 0; q < 5; ++q) S.H2[(7 + q) * n + c] = hh[1 + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) S.U2[q * n + c] = Un[q];
    if (!ok) return 0ull;
    const double rate = fmax((fabs(unx) + sn * CMAX) / P.dx, (fabs(uny) + sn * CMAX) / P.dy);
    return (unsigned long long)__double_as_longlong(rate);
}

// Launch bounds: FP32 168 registers (3 waves per SIMD); FP64 2 waves per SIMD, which
// spills about 290 B per lane and still runs 1.33x faster than 1 wave without spills.
// A cell still iterating after P.iter_split iterations (0: never) is handed to the tail
// kernel: its index, its iteration state (u_x, u_y, T and the frame one iteration back:
// 6 planes of tail_n R) and it | have_pp << 16 are appended to the list, whose length is
// tail_count[0] (cleared by dt_kernel); a full list leaves the cell here.
template <typename R, int REG, bool SPLIT>
__global__ __launch_bounds__(256, sizeof(R) == 4 ? 3 : 2) void sl_kernel_2d(Params P, State<R> S, int slot)
{
    __shared__ R L[Layout<2>::NL * SL2_NT];
    // FP32: per thread, the x weights of the 5 stencil columns (float4 of the 4 node columns)
    __shared__ float4 WX[sizeof(R) == 4 ? 5 * 256 : 1];
    const int tx = (int)blockIdx.x % ((P.nx + SL2_T - 1) / SL2_T);
    const int ty = (int)blockIdx.x / ((P.nx + SL2_T - 1) / SL2_T);
    const int i0 = tx * SL2_T, j0 = ty * SL2_T;
    // the tile: cells (i0 - 2 .. i0 + 17, j0 - 2 .. j0 + 17); slots outside the two ghost
    // layers belong to no stencil of a cell of the grid and are left unset
    for (int v = threadIdx.x; v < SL2_NT; v += blockDim.x) {
        const int i = i0 - 2 + v % SL2_W, j = j0 - 2 + v / SL2_W;
        if (i < -2 || i >= P.nx + 2 || j < -2 || j >= P.ny + 2) continue;
        const CellRef cr = map2d(P, i, j, S.tstart[0]);
        plus_record<2, R>(P, S, cr, 0.0, L + v, SL2_NT, 0);
    }
    __syncthreads();
    const int ci = i0 + (int)threadIdx.x % SL2_T, cj = j0 + (int)threadIdx.x / SL2_T;
    const bool active = ci < P.nx && cj < P.ny;
    const int64_t c = (int64_t)ci + (int64_t)P.nx * cj;
    const double dt = S.dt[0];
    const bool work = active && dt > 0.0;
    unsigned long long depout = 0ull, bits = 0ull;
    bool conv = false, handed = false;
    int iters = 0;
    if (work) {
        const int base = (int)threadIdx.x % SL2_T + SL2_W * ((int)threadIdx.x / SL2_T); // slot of (ci-2, cj-2)
        const int own = base + 2 + 2 * SL2_W;
        SlIter<R> I;
        I.ux = L[own];
        I.uy = L[SL2_NT + own];
        I.T = L[17 * SL2_NT + own];
        I.pux = R(0);
        I.puy = R(0);
        I.pT = R(1);
        I.have_pp = false;
        const R kx = (R)(dt / P.dx), ky = (R)(dt / P.dy);
        int code = SL_GO;
        for (I.it = 1; I.it <= P.max_iter; ++I.it) {
            code = sl_iterate<R, REG, false>(L, base, WX + threadIdx.x, nullptr, false, 0, 0, kx, ky, P.Cv, P.tol, I,
                                             depout);
            if (code != SL_GO) break;
            if (SPLIT && I.it == P.iter_split && I.it < P.max_iter) {
                // hand the cell over: one list slot per handing lane, one atomic per wave
                const unsigned long long m = __ballot(1);
                const int lead = __ffsll((long long)m) - 1;
                const int lane = (int)(threadIdx.x & 63);
                int start = 0;
                if (lane == lead) start = atomicAdd(S.tail_count, __popcll(m));
                start = __shfl(start, lead, 64);
                const int64_t e = (int64_t)start + __popcll(m & ((1ull << lane) - 1ull));
                if (e < P.tail_n) {
                    const int64_t tn = P.tail_n;
                    S.tail_f[e] = (int)c;
                    S.tail_meta[e] = I.it | (I.have_pp ? 1 << 16 : 0);
                    S.tail_s[e] = I.ux;
                    S.tail_s[tn + e] = I.uy;
                    S.tail_s[2 * tn + e] = I.T;
                    S.tail_s[3 * tn + e] = I.pux;
                    S.tail_s[4 * tn + e] = I.puy;
                    S.tail_s[5 * tn + e] = I.pT;
                    handed = true;
                    break;
                }
            }
        }
        iters = min(I.it, P.max_iter);
        if (!handed) {
            conv = code == SL_CONVERGED;
            bits = sl_finish<R>(P, S, c, dt, I);
        }
    } else if (active) {
        // a finished run keeps its state
        const int64_t n = P.ncell;
        for (int q = 0; q < Layout<2>::NH; ++q) S.H2[q * n + c] = S.H[q * n + c];
        for (int q = 0; q < 4; ++q) S.U2[q * n + c] = S.U[q * n + c];
    }
    const bool done = work && !handed;
    vmax_update<R>(P, S, slot ^ 1, 0, done, bits);
    stat_add4(S.stats, ST_FACES, done ? 1u : 0u, ST_NONCONV, (done && !conv) ? 1u : 0u, ST_CELLS,
              done ? 1u : 0u, ST_CONV_CELLS, (done && conv) ? 1u : 0u);
    stat_add32(S.stats, ST_ITERS, (unsigned)iters);
    stat_add32(S.stats, ST_DEPOUT, (unsigned)depout);
    stat_max32(S.stats, ST_ITMAX, done ? (unsigned)iters : 0u);
    if (depout) atomicOr(S.err, ERR_DEPART);
}

// the cells the SL kernel handed over, one per 32-lane group (two per wave): the group's
// lanes build the 25 stencil records of its cell once (they do not change within the
// step) and continue the cell's iteration from the saved state with the stencil spread
// over them (sl_advect_lanes_2d); the first lane finishes the cell as the SL kernel does.
// A fixed grid strides over the list; the trip count is uniform over each block.
constexpr int SL2_TAIL_BLOCKS = 1024;

template <typename R, int REG>
__global__ __launch_bounds__(64) void sl_tail_kernel_2d(Params P, State<R> S, int slot)
{
    const int64_t n = min((int64_t)S.tail_count[0], P.tail_n);
    const double dt = S.dt[0];
    const R kx = (R)(dt / P.dx), ky = (R)(dt / P.dy);
    const int lane = (int)(threadIdx.x & 31), grp = (int)(threadIdx.x >> 5);
    const int a = lane % 5, b = lane / 5;
    const bool mine = lane < 25;
    for (int64_t e0 = 2 * (int64_t)blockIdx.x; e0 < n; e0 += 2 * (int64_t)gridDim.x) {
        const int64_t e = e0 + grp;
        const bool has = e < n; // uniform over the group
        unsigned long long depout = 0ull, bits = 0ull;
        bool conv = false;
        int iters = 0, it0 = 0;
        if (has) {
            const int64_t tn = P.tail_n;
            const int64_t c = S.tail_f[e];
            const int meta = S.tail_meta[e];
            SlIter<R> I;
            I.ux = S.tail_s[e];
            I.uy = S.tail_s[tn + e];
            I.T = S.tail_s[2 * tn + e];
            I.pux = S.tail_s[3 * tn + e];
            I.puy = S.tail_s[4 * tn + e];
            I.pT = S.tail_s[5 * tn + e];
            I.have_pp = (meta >> 16) & 1;
            it0 = meta & 0xffff;
            const int ci = (int)(c % P.nx), cj = (int)(c / P.nx);
            R rec[Layout<2>::NL];
            if (mine) {
                const CellRef cr = map2d(P, ci - 2 + a, cj - 2 + b, S.tstart[0]);
                plus_record<2, R>(P, S, cr, 0.0, rec, 1, 0);
            }
            int code = SL_GO;
            for (I.it = it0 + 1; I.it <= P.max_iter; ++I.it) {
                code = sl_iterate<R, REG, true>(nullptr, 0, nullptr, rec, mine, a, b, kx, ky, P.Cv, P.tol, I, depout);
                if (code != SL_GO) break;
            }
            iters = min(I.it, P.max_iter);
            conv = code == SL_CONVERGED;
            if (lane == 0) bits = sl_finish<R>(P, S, c, dt, I);
        }
        const bool lead = has && lane == 0;
        if (!lead) {
            depout = 0ull;
            iters = it0 = 0;
        }
        vmax_update<R>(P, S, slot ^ 1, 0, lead, bits);
        stat_add4(S.stats, ST_FACES, lead ? 1u : 0u, ST_NONCONV, (lead && !conv) ? 1u : 0u, ST_CELLS,
                  lead ? 1u : 0u, ST_CONV_CELLS, (lead && conv) ? 1u : 0u);
        stat_add32(S.stats, ST_ITERS, (unsigned)(iters - it0));
        stat_add32(S.stats, ST_DEPOUT, (unsigned)depout);
        stat_max32(S.stats, ST_ITMAX, (unsigned)iters);
        if (depout) atomicOr(S.err, ERR_DEPART);
    }
}

} // namespace pond
