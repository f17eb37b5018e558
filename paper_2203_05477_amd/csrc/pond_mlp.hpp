// pond_mlp.hpp -- learned seed of the face-frame iteration: a 2 x 64 hidden-layer MLP run
// with BF16 MFMA (v_mfma_f32_16x16x32_bf16) and FP32 accumulation.
//
// Input of one face (64 values, FP32 in memory, BF16 at the MFMA): the 3 x 3 cells centred
// on the face's lower neighbour (west for x-faces, south for y-faces) at the start of the
// step, each as log(rho/rho_c), (u_n - u_cn)/s_c, (u_t - u_ct)/s_c, log(T/T_c) in the face's
// normal/tangential coordinates (s_c = sqrt T_c of the centre cell), then the previous face
// frame (the plain seed) in the same normalized form and a flag telling whether it exists;
// the rest is zero. Output (3): the converged face frame in the same normalized form, as a
// correction to the plain seed when the face has one (the seed is then plain + output).
// A y-face is presented as an x-face with the axes exchanged, so one network serves both;
// 1D faces see their 3 cells as a y-uniform stencil.
//
// Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3 with W1, W2 64 x 64,
// W3 3 x 64. Parameter vector (FP32 master copy): W1 (row-major, out x in), b1, W2, b2,
// W3, b3 = 8515 values. The network only seeds the predictor-corrector; the iteration still
// runs to the same tolerance.
//
// MFMA operand layouts for 16x16x32 (lane l, group g = l / 16, column c = l % 16):
//   A (16 x 32): lane holds A[c][8g .. 8g+7];  B (32 x 16): lane holds B[8g .. 8g+7][c];
//   D (16 x 16): lane holds D[4g + i][c], i = 0..3.
// Chaining layers in registers: the forward pass computes h^T = W x^T tile by tile, so a
// lane holds hidden units 16t + 4g + i of sample c. Taken from tiles 2k and 2k+1, those 8
// values are exactly a B operand of k-block k if the hidden units of that block are ordered
// (t = 2k: 4g + j; t = 2k+1: 16 + 4g + j - 4); the weights of the next layer are read in
// that order, so no activation ever goes through LDS in the forward pass.
#pragma once

#include <hip/hip_runtime.h>

#include "pond_kernels.hpp"

namespace pond {

constexpr int MLP_IN = 64, MLP_H = 64, MLP_OUT = 3;
constexpr int MLP_NF = 40; // features actually used (36 stencil + 3 seed + 1 flag)
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H,
              OFF_B2 = OFF_W2 + MLP_H * MLP_H, OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_OUT * MLP_H,
              MLP_NPARAM = OFF_B3 + MLP_OUT;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

PD f4 mfma16(bf16x8 a, bf16x8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// hidden unit of position j (0..7) of lane group g in k-block kb (register chaining order)
PD int chain_unit(int kb, int g, int j) { return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4)); }

struct MlpDevice {
    bool ready = false;
    float *master = nullptr;     // MLP_NPARAM FP32
    float *adam_m = nullptr, *adam_v = nullptr;
    __bf16 *wbf = nullptr;       // BF16 copies: W1 (64x64), W2 (64x64), W3 padded (16x64)
    float *partial = nullptr;    // per-wave partial gradients (+ loss)
    float *grad = nullptr;       // reduced gradient (+ loss)
    int npartial = 0;
    int adam_t = 0;
    // seed selection
    int *list = nullptr;         // face ids whose seed the network sets
    int *count = nullptr;
    int64_t list_cap = 0;
    int hard_iters = 2;          // faces that took at least this many iterations last step
};

// ---------------------------------------------------------------------------------
// features of one face
// ---------------------------------------------------------------------------------

// primitive state of a (possibly ghost) cell for the features: rho, u (x, y), T
template <int D>
PD void feat_cell(const Params &P, const double *U, const CellRef &c, double &rho, double u[2], double &T)
{
    if (c.src < 0) {
        double st[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) st[q] = c.falt ? P.bc_alt[c.fside][q] : P.bc_state[c.fside][q];
        rho = st[0];
        u[0] = st[1];
        u[1] = D == 2 ? st[2] : 0.0;
        T = st[3] / st[0];
    } else {
        prim<D>(U, P.ncell, c.src, rho, u, T, P.Cv);
        if (c.mx) u[0] = -u[0];
        if (c.my) u[1] = -u[1];
    }
}

// x[64] (zero padded) and ref[4] = (u_cn, u_ct, s_c, T_c) of face f; axis 0 in 1D.
// Seed frame taken from the face state planes F (previous face frame).
template <int D, typename R>
PD void face_features(const Params &P, const State<R> &S, int64_t f, float *x, float *ref)
{
    int axis = 0, ci = 0, cj = 0;
    int64_t tube_off = 0;
    int tube_n = 0, k = 0;
    if (D == 1) {
        k = S.face_inst ? S.face_inst[f] : 0;
        tube_off = S.cell_off[k];
        tube_n = (int)(S.cell_off[k + 1] - tube_off);
        ci = (int)(f - (tube_off + k)) - 1; // lower neighbour (local index)
    } else if (f < P.nfx) {
        ci = (int)(f % (P.nx + 1)) - 1;
        cj = (int)(f / (P.nx + 1));
    } else {
        axis = 1;
        int64_t q = f - P.nfx;
        ci = (int)(q % P.nx);
        cj = (int)(q / P.nx) - 1;
    }
    const double t = S.tstart[k];
    double rc, uc[2], Tc;
    double cells[9][4];
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
            int ii, jj;
            if (D == 1) {
                ii = ci + a;
                jj = 0;
            } else if (axis == 0) {
                ii = ci + a;
                jj = cj + b;
            } else {
                ii = ci + b;
                jj = cj + a;
            }
            CellRef c{0, 0, 0, -1, 0};
            if (D == 1) {
                if (ii >= 0 && ii < tube_n) {
                    c.src = tube_off + ii;
                } else {
                    int side = ii < 0 ? 0 : 1;
                    int sq = side_rule(P, side, ii, tube_n, 0.0, 0.0, 0.0, t, c.mx, c.fside, c.falt);
                    c.src = sq < 0 ? -1 : tube_off + sq;
                }
            } else {
                c = map2d(P, ii, jj, t);
            }
            double rho, u[2], T;
            feat_cell<D>(P, S.U, c, rho, u, T);
            const int e = (a + 1) * 3 + (b + 1);
            cells[e][0] = rho;
            cells[e][1] = axis ? u[1] : u[0]; // normal
            cells[e][2] = axis ? u[0] : u[1]; // tangential
            cells[e][3] = T;
        }
    rc = cells[4][0];
    uc[0] = cells[4][1];
    uc[1] = cells[4][2];
    Tc = cells[4][3];
    // logarithms of ratios in FP32 (hardware log): the features feed a BF16 network
    const double sc = sqrt(Tc), isc = 1.0 / sc, irc = 1.0 / rc, iTc = 1.0 / Tc;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        x[4 * e + 0] = __logf((float)(cells[e][0] * irc));
        x[4 * e + 1] = (float)((cells[e][1] - uc[0]) * isc);
        x[4 * e + 2] = (float)((cells[e][2] - uc[1]) * isc);
        x[4 * e + 3] = __logf((float)(cells[e][3] * iTc));
    }
    const int64_t nf = P.nface;
    double su[2], sT;
    if (D == 1) {
        su[0] = (double)S.F[f];
        su[1] = 0.0;
        sT = (double)S.F[nf + f];
    } else {
        su[0] = (double)S.F[(axis ? 1 : 0) * nf + f];
        su[1] = (double)S.F[(axis ? 0 : 1) * nf + f];
        sT = (double)S.F[2 * nf + f];
    }
    if (sT > 0.0) {
        x[36] = (float)((su[0] - uc[0]) * isc);
        x[37] = (float)((su[1] - uc[1]) * isc);
        x[38] = __logf((float)(sT * iTc));
        x[39] = 1.0f;
    } else {
        x[36] = x[37] = x[38] = x[39] = 0.0f;
    }
    for (int q = MLP_NF; q < MLP_IN; ++q) x[q] = 0.0f;
    ref[0] = (float)uc[0];
    ref[1] = (float)uc[1];
    ref[2] = (float)sc;
    ref[3] = (float)Tc;
    (void)rc;
}

// features of all faces (or of the faces listed in `list`, count `*count`)
template <int D, typename R>
__global__ void mlp_features_kernel(Params P, State<R> S, float *X, float *ref)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.nface) return;
    face_features<D, R>(P, S, f, X + f * MLP_IN, ref + f * 4);
}

// targets: the current face frames normalized by the references of the features, minus
// the normalized previous frame (the plain seed) when the face had one -- the network
// learns the correction to the plain seed
template <int D, typename R>
__global__ void mlp_targets_kernel(Params P, State<R> S, const float *X, const float *ref, float *Y)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= P.nface) return;
    const int64_t nf = P.nface;
    int axis = (D == 2 && f >= P.nfx) ? 1 : 0;
    double un, ut, T;
    if (D == 1) {
        un = S.F[f];
        ut = 0.0;
        T = S.F[nf + f];
    } else {
        un = S.F[(axis ? 1 : 0) * nf + f];
        ut = S.F[(axis ? 0 : 1) * nf + f];
        T = S.F[2 * nf + f];
    }
    const float *r = ref + f * 4;
    const float *x = X + f * MLP_IN;
    const float has = x[39];
    Y[f * 4 + 0] = (float)((un - r[0]) / r[2]) - has * x[36];
    Y[f * 4 + 1] = (float)((ut - r[1]) / r[2]) - has * x[37];
    Y[f * 4 + 2] = (float)log(T / (double)r[3]) - has * x[38];
    Y[f * 4 + 3] = 0.0f;
}

// ---------------------------------------------------------------------------------
// forward pass of one 16-sample tile held as B operands (register chaining)
// ---------------------------------------------------------------------------------

struct MlpRegs {
    bf16x8 w1[4][2], w2[4][2], w3[2];
    float b1[4][4], b2[4][4], b3[4];
};

PD void mlp_load_regs(const __bf16 *wbf, const float *master, MlpRegs &W)
{
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const __bf16 *W1 = wbf, *W2 = wbf + MLP_H * MLP_IN, *W3 = wbf + 2 * MLP_H * MLP_IN;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                W.w1[t][kb][j] = W1[(16 * t + c) * MLP_IN + 32 * kb + 8 * g + j];
                W.w2[t][kb][j] = W2[(16 * t + c) * MLP_H + chain_unit(kb, g, j)];
            }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) W.w3[kb][j] = W3[c * MLP_H + chain_unit(kb, g, j)];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            W.b1[t][i] = master[OFF_B1 + 16 * t + 4 * g + i];
            W.b2[t][i] = master[OFF_B2 + 16 * t + 4 * g + i];
        }
#pragma unroll
    for (int i = 0; i < 4; ++i) W.b3[i] = (4 * g + i < MLP_OUT) ? master[OFF_B3 + 4 * g + i] : 0.0f;
}

// xb[kb]: features 32 kb + 8 g .. +7 of sample c. Returns the outputs 4g+i of sample c;
// optionally the hidden activations (post-relu, FP32) in the chained tile layout.
PD f4 mlp_tile_forward(const MlpRegs &W, const bf16x8 xb[2], f4 h1o[4], f4 h2o[4])
{
    f4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f4 a = {0.f, 0.f, 0.f, 0.f};
        a = mfma16(W.w1[t][0], xb[0], a);
        a = mfma16(W.w1[t][1], xb[1], a);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = fmaxf(a[i] + W.b1[t][i], 0.0f);
        h1[t] = a;
    }
    bf16x8 hb[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hb[kb][j] = (__bf16)h1[2 * kb][j];
            hb[kb][4 + j] = (__bf16)h1[2 * kb + 1][j];
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f4 a = {0.f, 0.f, 0.f, 0.f};
        a = mfma16(W.w2[t][0], hb[0], a);
        a = mfma16(W.w2[t][1], hb[1], a);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = fmaxf(a[i] + W.b2[t][i], 0.0f);
        h2[t] = a;
    }
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            hb[kb][j] = (__bf16)h2[2 * kb][j];
            hb[kb][4 + j] = (__bf16)h2[2 * kb + 1][j];
        }
    f4 y = {0.f, 0.f, 0.f, 0.f};
    y = mfma16(W.w3[0], hb[0], y);
    y = mfma16(W.w3[1], hb[1], y);
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] += W.b3[i];
    if (h1o)
#pragma unroll
        for (int t = 0; t < 4; ++t) h1o[t] = h1[t];
    if (h2o)
#pragma unroll
        for (int t = 0; t < 4; ++t) h2o[t] = h2[t];
    return y;
}

PD void load_xb(const float *X, int64_t n, int64_t s0, bf16x8 xb[2])
{
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const int64_t s = s0 + c;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) xb[kb][j] = (__bf16)(s < n ? X[s * MLP_IN + 32 * kb + 8 * g + j] : 0.0f);
}

// inference: Y[n][4] (outputs 0..2) from X[n][64]; one wave per 16-sample tile, grid-stride
__global__ __launch_bounds__(64) void mlp_forward_kernel(const __bf16 *wbf, const float *master,
                                                         const float *X, int64_t n, float *Y)
{
    MlpRegs W;
    mlp_load_regs(wbf, master, W);
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    for (int64_t s0 = (int64_t)blockIdx.x * 16; s0 < n; s0 += (int64_t)gridDim.x * 16) {
        bf16x8 xb[2];
        load_xb(X, n, s0, xb);
        f4 y = mlp_tile_forward(W, xb, nullptr, nullptr);
        const int64_t s = s0 + c;
        if (g == 0 && s < n)
#pragma unroll
            for (int i = 0; i < 4; ++i) Y[s * 4 + i] = (i < MLP_OUT) ? y[i] : 0.0f;
    }
}

// ---------------------------------------------------------------------------------
// training: forward + backward per 32-sample chunk, per-wave partial gradients
// ---------------------------------------------------------------------------------

// loss = (1/n) sum_s sum_o (y - t)^2. One wave per block; LDS per wave: X, H1, H2 (bf16),
// masks of z1 > 0, z2 > 0, dZ1, dZ2 (bf16), dY (fp32).
struct TrainLds {
    __bf16 X[32][MLP_IN];
    __bf16 H1[32][MLP_H];
    __bf16 H2[32][MLP_H];
    __bf16 D1[32][MLP_H]; // dZ1
    __bf16 D2[32][MLP_H]; // dZ2
    unsigned char M1[32][MLP_H], M2[32][MLP_H];
    float dY[32][4];
};

__global__ __launch_bounds__(64) void mlp_train_kernel(const __bf16 *wbf, const float *master,
                                                       const float *X, const float *Yt, int64_t n,
                                                       float *partial)
{
    __shared__ TrainLds S;
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    MlpRegs W;
    mlp_load_regs(wbf, master, W);
    const __bf16 *W2 = wbf + MLP_H * MLP_IN, *W3 = wbf + 2 * MLP_H * MLP_IN;
    f4 gW1[4][4], gW2[4][4], gW3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW3[a] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW1[a][b] = gW2[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, loss = 0.f; // lane l: unit l (b1, b2), output l (b3)
    const float inv_n = 1.0f / (float)n;
    for (int64_t base = (int64_t)blockIdx.x * 32; base < n; base += (int64_t)gridDim.x * 32) {
        // ---- forward of the two 16-sample tiles; keep activations in LDS ----
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int64_t s0 = base + 16 * half;
            bf16x8 xb[2];
            load_xb(X, n, s0, xb);
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int j = 0; j < 8; ++j) S.X[16 * half + c][32 * kb + 8 * g + j] = xb[kb][j];
            f4 h1[4], h2[4];
            f4 y = mlp_tile_forward(W, xb, h1, h2);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int u = 16 * t + 4 * g + i, s = 16 * half + c;
                    S.H1[s][u] = (__bf16)h1[t][i];
                    S.H2[s][u] = (__bf16)h2[t][i];
                    S.M1[s][u] = h1[t][i] > 0.0f;
                    S.M2[s][u] = h2[t][i] > 0.0f;
                }
            const int64_t s = s0 + c;
            if (g == 0)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float d = 0.0f;
                    if (i < MLP_OUT && s < n) {
                        float e = y[i] - Yt[s * 4 + i];
                        loss += e * e;
                        d = 2.0f * e * inv_n;
                    }
                    S.dY[16 * half + c][i] = d;
                }
        }
        __syncthreads();
        // ---- layer 3: gW3 += dY^T H2 (MFMA, K = 32 samples); db3 ----
        {
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)((c < MLP_OUT) ? S.dY[8 * g + j][c] : 0.0f);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = S.H2[8 * g + j][16 * t + c];
                gW3[t] = mfma16(a, b, gW3[t]);
            }
            if (l < MLP_OUT)
                for (int s = 0; s < 32; ++s) gb3 += S.dY[s][l];
        }
        // ---- dZ2 = (dY W3) * [z2 > 0]  (K = 3: vector ALU) ----
        for (int e = l; e < 32 * MLP_H; e += 64) {
            const int s = e / MLP_H, u = e % MLP_H;
            float d = 0.0f;
#pragma unroll
            for (int o = 0; o < MLP_OUT; ++o) d += S.dY[s][o] * (float)W3[o * MLP_H + u];
            S.D2[s][u] = (__bf16)(S.M2[s][u] ? d : 0.0f);
        }
        __syncthreads();
        // ---- layer 2: gW2 += dZ2^T H1; db2; dZ1 = (dZ2 W2) * [z1 > 0] ----
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = S.D2[8 * g + j][16 * ot + c];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = S.H1[8 * g + j][16 * kt + c];
                gW2[ot][kt] = mfma16(a, b, gW2[ot][kt]);
            }
        }
        for (int s = 0; s < 32; ++s) gb2 += (float)S.D2[s][l];
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    bf16x8 a, b;
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        a[j] = S.D2[16 * st + c][32 * kb + 8 * g + j];
                        b[j] = W2[(32 * kb + 8 * g + j) * MLP_H + 16 * kt + c];
                    }
                    acc = mfma16(a, b, acc);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int s = 16 * st + 4 * g + i, u = 16 * kt + c;
                    S.D1[s][u] = (__bf16)(S.M1[s][u] ? acc[i] : 0.0f);
                }
            }
        __syncthreads();
        // ---- layer 1: gW1 += dZ1^T X; db1 ----
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = S.D1[8 * g + j][16 * ot + c];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = S.X[8 * g + j][16 * kt + c];
                gW1[ot][kt] = mfma16(a, b, gW1[ot][kt]);
            }
        }
        for (int s = 0; s < 32; ++s) gb1 += (float)S.D1[s][l];
        __syncthreads();
    }
    // ---- per-wave partial gradient in the parameter layout, loss in the last slot ----
    float *P = partial + (size_t)blockIdx.x * (MLP_NPARAM + 1);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = 16 * ot + 4 * g + i, k = 16 * kt + c;
                P[OFF_W1 + o * MLP_IN + k] = gW1[ot][kt][i];
                P[OFF_W2 + o * MLP_H + k] = gW2[ot][kt][i];
            }
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 4 * g + i, k = 16 * kt + c;
            if (o < MLP_OUT) P[OFF_W3 + o * MLP_H + k] = gW3[kt][i];
        }
    P[OFF_B1 + l] = gb1;
    P[OFF_B2 + l] = gb2;
    if (l < MLP_OUT) P[OFF_B3 + l] = gb3;
    // loss: sum over lanes
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (l == 0) P[MLP_NPARAM] = loss * inv_n;
}

// deterministic sum of the per-wave partials
__global__ void mlp_reduce_kernel(const float *partial, int nw, float *grad)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MLP_NPARAM) return;
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += partial[(size_t)w * (MLP_NPARAM + 1) + p];
    grad[p] = s;
}

// Adam on the FP32 master weights; refresh the BF16 copies
__global__ void mlp_adam_kernel(float *master, float *m, float *v, const float *grad, __bf16 *wbf,
                                float lr, float b1, float b2, float eps, int t)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gp = grad[p];
    const float mp = b1 * m[p] + (1.0f - b1) * gp;
    const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const float mh = mp / (1.0f - powf(b1, (float)t)), vh = vp / (1.0f - powf(b2, (float)t));
    const float w = master[p] - lr * mh / (sqrtf(vh) + eps);
    master[p] = w;
    if (p < OFF_B1)
        wbf[p] = (__bf16)w;
    else if (p >= OFF_W2 && p < OFF_B2)
        wbf[MLP_H * MLP_IN + (p - OFF_W2)] = (__bf16)w;
    else if (p >= OFF_W3 && p < OFF_B3)
        wbf[2 * MLP_H * MLP_IN + (p - OFF_W3)] = (__bf16)w;
}

// BF16 copies from the master weights (rows 3..15 of the padded W3 stay zero)
__global__ void mlp_pack_kernel(const float *master, __bf16 *wbf)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_H * MLP_IN) {
        wbf[p] = (__bf16)master[OFF_W1 + p];
        wbf[MLP_H * MLP_IN + p] = (__bf16)master[OFF_W2 + p];
    }
    if (p < 16 * MLP_H) wbf[2 * MLP_H * MLP_IN + p] = (p < MLP_OUT * MLP_H) ? (__bf16)master[OFF_W3 + p] : (__bf16)0.0f;
}

// ---------------------------------------------------------------------------------
// learned seed inside the step
// ---------------------------------------------------------------------------------

// Per-slot capacity of a list that the waves of a launch over n items (64 per wave) append
// to: each wave appends to the sub-list of its slot (wave_slot), so that no counter is hit
// by more than a handful of waves.
inline int64_t slot_cap(int64_t n)
{
    const int64_t waves = 4 * ((n + 255) / 256); // 256-thread blocks
    return 64 * ((waves + NSLOT - 1) / NSLOT);
}

// faces that took at least `hard` iterations in the previous step (or did not converge)
template <typename R>
__global__ void mlp_select_kernel(Params P, State<R> S, int hard, int *list, int *count, int cap)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool take = false;
    if (f < P.nface) {
        const int k = S.face_inst ? S.face_inst[f] : 0;
        const int v = S.fiter[f];
        take = (S.dt[k] > 0.0) && (((v & 0xffff) >= hard) || ((v >> 16) & 1));
    }
    // wave-aggregated append to the wave's sub-list
    unsigned long long m = __ballot(take);
    int nt = __popcll(m);
    int base = 0;
    const int lane = threadIdx.x & 63;
    const unsigned slot = wave_slot();
    if (lane == 0 && nt) base = atomicAdd(&count[slot], nt);
    base = __shfl(base, 0, 64);
    const int pos = base + __popcll(m & ((1ull << lane) - 1ull));
    if (take && pos < cap) list[(int64_t)slot * cap + pos] = (int)f;
}

// features + network + seed write for the listed faces; one wave per 64 faces. The
// faces of the NSLOT sub-lists, concatenated, are dealt out 16 per block in turn (the hard
// faces cluster in the sub-lists of the waves that cover a shock).
template <int D, typename R>
__global__ __launch_bounds__(64) void mlp_seed_kernel(Params P, State<R> S, const __bf16 *wbf,
                                                      const float *master, const int *lists,
                                                      const int *counts, int cap)
{
    __shared__ float xs[64][MLP_IN + 1];
    __shared__ float rs[64][4];
    __shared__ int pre[NSLOT + 1];
    const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    {
        // pre[s] = listed faces in the sub-lists before s; lane l sums sub-lists 4l..4l+3
        static_assert(NSLOT == 256, "4 sub-lists per lane of a 64-lane block");
        int v[4], x = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = min(counts[4 * l + q], cap);
            x += v[q];
        }
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (l >= d) x += y;
        }
        int run = x - (v[0] + v[1] + v[2] + v[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pre[4 * l + q] = run;
            run += v[q];
        }
        if (l == 63) pre[NSLOT] = x;
        __syncthreads();
    }
    const int n = pre[NSLOT];
    if ((int)blockIdx.x * 64 >= n) return;
    MlpRegs W;
    mlp_load_regs(wbf, master, W);
    // list index of the k-th listed face: in the last sub-list s with pre[s] <= k
    auto entry = [&](int k) {
        int lo = 0, hi = NSLOT - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= k)
                lo = mid;
            else
                hi = mid - 1;
        }
        return (int64_t)lo * cap + (k - pre[lo]);
    };
    const int64_t nf = P.nface;
    for (int t0 = (int)blockIdx.x * 64; t0 < n; t0 += (int)gridDim.x * 64) {
        // every lane gathers the features of one face, then 4 tiles of 16 faces go through
        // the network
        if (t0 + l < n) {
            float x[MLP_IN], ref[4];
            face_features<D, R>(P, S, lists[entry(t0 + l)], x, ref);
            for (int q = 0; q < MLP_IN; ++q) xs[l][q] = x[q];
            for (int q = 0; q < 4; ++q) rs[l][q] = ref[q];
        } else {
            for (int q = 0; q < MLP_IN; ++q) xs[l][q] = 0.0f;
            rs[l][0] = rs[l][1] = 0.0f;
            rs[l][2] = rs[l][3] = 1.0f;
        }
        __syncthreads();
#pragma unroll 1
        for (int tile = 0; tile < 4; ++tile) {
            const int fc = 16 * tile + c; // face of this lane's column in the tile
            bf16x8 xb[2];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int j = 0; j < 8; ++j) xb[kb][j] = (__bf16)xs[fc][32 * kb + 8 * g + j];
            f4 y = mlp_tile_forward(W, xb, nullptr, nullptr);
            if (g == 0 && t0 + fc < n) {
                const int64_t f = lists[entry(t0 + fc)];
                const int axis = (D == 2 && f >= P.nfx) ? 1 : 0;
                const float *r = rs[fc];
                const float has = xs[fc][39];
                const float y0 = y[0] + has * xs[fc][36], y1 = y[1] + has * xs[fc][37];
                const float y2 = y[2] + has * xs[fc][38];
                const double un = r[0] + (double)r[2] * y0;
                const double ut = r[1] + (double)r[2] * y1;
                const double T = (double)r[3] * exp((double)fminf(fmaxf(y2, -20.0f), 20.0f));
                if (D == 1) {
                    S.F[f] = (R)un;
                    S.F[nf + f] = (R)T;
                } else {
                    S.F[(axis ? 1 : 0) * nf + f] = (R)un;
                    S.F[(axis ? 0 : 1) * nf + f] = (R)ut;
                    S.F[2 * nf + f] = (R)T;
                }
            }
        }
        __syncthreads();
    }
}

inline void mlp_free(MlpDevice &M)
{
    void *ptrs[] = {M.master, M.adam_m, M.adam_v, M.wbf, M.partial, M.grad, M.list, M.count};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    M = MlpDevice();
}

template <int D, typename R>
hipError_t mlp_seed_launch(const MlpDevice &M, const Params &P, const State<R> &S, hipStream_t st)
{
    // M.count is cleared by the step's dt_kernel (State::seed_count)
    const int cap = (int)slot_cap(P.nface);
    mlp_select_kernel<R><<<(unsigned)((P.nface + 255) / 256), 256, 0, st>>>(P, S, M.hard_iters, M.list, M.count, cap);
    mlp_seed_kernel<D, R><<<NSLOT * 4, 64, 0, st>>>(P, S, M.wbf, M.master, M.list, M.count, cap);
    return hipGetLastError();
}

} // namespace pond
