// pond_core.hpp -- device arithmetic of the PonD step on gfx950.
//
// Every cell, face or stencil distribution is held as Hermite coefficients h in its own
// frame lambda = {u, T} (s = sqrt T): f_i = W_i sum_{p,q} h[p][q] He_p(c_ix) He_q(c_iy),
// the tensor-product form of the Grad expansion of Sec. II.C (h10 = a_x, h20 = a_xx/2,
// h11 = a_xy, h30 = a_xxx/6, h21 = a_xxy/2, ...; in 1D h_p = a_p/p!). A change of frame
// lambda -> lambda' is computed on the dimensionless raw moments mu[k][l] = sum f c_x^k c_y^l:
// with r = s/s' and d = (u - u')/s', the moments in lambda' are those of (r c + d), a
// binomial shift. Because Grad's projection is fixed by M_0..M_3 (M_0..M_2 for g), this is
// the paper's regularized transformation written in frame-relative variables: no quantity
// of size u^3 is ever formed, so FP32 keeps its relative accuracy at any Mach number.
//
// Coefficient order. 2D, degree <= 3: 00 10 01 20 11 02 30 21 12 03 (10 values);
// degree <= 2: the first 6. 1D: h0 h1 h2 h3.
// Population order: i = ix + 4 iy, nodes ascending: -cb, -ca, +ca, +cb (Table I, D1Q4).
#pragma once

#include <hip/hip_runtime.h>

#define PD __device__ __forceinline__

namespace pond {

// D1Q4 (Table I): nodes +-sqrt(3 -+ sqrt 6), weights (3 +- sqrt 6)/12, and the
// probabilists' Hermite polynomials He2 = c^2 - 1, He3 = c^3 - 3c at the positive nodes.
template <typename R>
struct Lat {
    static constexpr R ca = R(7.41963784302725803954e-01);
    static constexpr R cb = R(2.33441421833897733151e+00);
    static constexpr R wa = R(4.54124145231931508615e-01);
    static constexpr R wb = R(4.58758547680684913850e-02);
    static constexpr R he2a = R(-4.49489742783178103380e-01);
    static constexpr R he2b = R(4.44948974278317788134e+00);
    static constexpr R he3a = R(-1.81743267916611750401e+00);
    static constexpr R he3b = R(5.71812368322853536995e+00);
};

template <typename R>
PD R node(int k)
{
    // k = 0..3 -> -cb, -ca, +ca, +cb
    R c = (k == 1 || k == 2) ? Lat<R>::ca : Lat<R>::cb;
    return (k < 2) ? -c : c;
}

template <typename R>
PD R weight1(int k)
{
    return (k == 1 || k == 2) ? Lat<R>::wa : Lat<R>::wb;
}

constexpr double CMAX = 2.33441421833897733151e+00; // largest |node|

// ---------------------------------------------------------------------------------
// Hermite coefficients <-> raw dimensionless moments (Gauss-Hermite is exact here)
// ---------------------------------------------------------------------------------

template <typename R>
PD void h2mu_1d(const R h[4], R mu[4])
{
    mu[0] = h[0];
    mu[1] = h[1];
    mu[2] = h[0] + R(2) * h[2];
    mu[3] = R(3) * h[1] + R(6) * h[3];
}

template <typename R>
PD void mu2h_1d(const R mu[4], R h[4])
{
    h[0] = mu[0];
    h[1] = mu[1];
    h[2] = R(0.5) * (mu[2] - mu[0]);
    h[3] = (mu[3] - R(3) * mu[1]) * R(1.0 / 6.0);
}

// 2D, order 3 (10) -- the first 6 entries are the order-2 set
template <typename R>
PD void h2mu_2d(const R h[10], R mu[10], int n)
{
    mu[0] = h[0];
    mu[1] = h[1];
    mu[2] = h[2];
    mu[3] = h[0] + R(2) * h[3];
    mu[4] = h[4];
    mu[5] = h[0] + R(2) * h[5];
    if (n > 6) {
        mu[6] = R(3) * h[1] + R(6) * h[6];
        mu[7] = h[2] + R(2) * h[7];
        mu[8] = h[1] + R(2) * h[8];
        mu[9] = R(3) * h[2] + R(6) * h[9];
    }
}

template <typename R>
PD void mu2h_2d(const R mu[10], R h[10], int n)
{
    h[0] = mu[0];
    h[1] = mu[1];
    h[2] = mu[2];
    h[3] = R(0.5) * (mu[3] - mu[0]);
    h[4] = mu[4];
    h[5] = R(0.5) * (mu[5] - mu[0]);
    if (n > 6) {
        h[6] = (mu[6] - R(3) * mu[1]) * R(1.0 / 6.0);
        h[7] = R(0.5) * (mu[7] - mu[2]);
        h[8] = R(0.5) * (mu[8] - mu[1]);
        h[9] = (mu[9] - R(3) * mu[2]) * R(1.0 / 6.0);
    }
}

// moments of (r c + d) from moments of c: 1D, degree 3 (n = 4) or 2 (n = 3)
template <typename R>
PD void shift_1d(R mu[4], R r, R d, int n)
{
    R r2 = r * r;
    R m1 = r * mu[1], m2 = r2 * mu[2];
    R m0 = mu[0];
    if (n > 3) {
        R m3 = r2 * r * mu[3];
        mu[3] = m3 + d * (R(3) * m2 + d * (R(3) * m1 + d * m0));
    }
    mu[2] = m2 + d * (R(2) * m1 + d * m0);
    mu[1] = m1 + d * m0;
}

// 2D binomial shift: x' = r c + d, moments up to total degree 3 (n = 10) or 2 (n = 6)
template <typename R>
PD void shift_2d(R mu[10], R r, R dx, R dy, int n)
{
    R r2 = r * r;
    // scale by r^(k+l)
    R v00 = mu[0], v10 = r * mu[1], v01 = r * mu[2];
    R v20 = r2 * mu[3], v11 = r2 * mu[4], v02 = r2 * mu[5];
    R v30 = R(0), v21 = R(0), v12 = R(0), v03 = R(0);
    if (n > 6) {
        R r3 = r2 * r;
        v30 = r3 * mu[6];
        v21 = r3 * mu[7];
        v12 = r3 * mu[8];
        v03 = r3 * mu[9];
    }
    // shift in x
    R c30 = v30 + dx * (R(3) * v20 + dx * (R(3) * v10 + dx * v00));
    R c20 = v20 + dx * (R(2) * v10 + dx * v00);
    R c10 = v10 + dx * v00;
    R c21 = v21 + dx * (R(2) * v11 + dx * v01);
    R c11 = v11 + dx * v01;
    R c12 = v12 + dx * v02;
    // shift in y
    mu[1] = c10;
    mu[2] = v01 + dy * v00;
    mu[3] = c20;
    mu[4] = c11 + dy * c10;
    mu[5] = v02 + dy * (R(2) * v01 + dy * v00);
    if (n > 6) {
        mu[6] = c30;
        mu[7] = c21 + dy * c20;
        mu[8] = c12 + dy * (R(2) * c11 + dy * c10);
        mu[9] = v03 + dy * (R(3) * v02 + dy * (R(3) * v01 + dy * v00));
    }
}

// ---------------------------------------------------------------------------------
// reduced populations p_i = f_i / W_i from Hermite coefficients
// ---------------------------------------------------------------------------------

template <typename R>
PD void eval_1d(const R h[4], R p[4], int order)
{
    R h3 = (order > 2) ? h[3] : R(0);
    R Ea = h[0] + h[2] * Lat<R>::he2a, Oa = h[1] * Lat<R>::ca + h3 * Lat<R>::he3a;
    R Eb = h[0] + h[2] * Lat<R>::he2b, Ob = h[1] * Lat<R>::cb + h3 * Lat<R>::he3b;
    p[0] = Eb - Ob;
    p[1] = Ea - Oa;
    p[2] = Ea + Oa;
    p[3] = Eb + Ob;
}

// 2D: sum factorization over y then x, with the parity of He_p at +-c
template <typename R>
PD void eval_2d(const R h[10], R p[16], int order)
{
    const bool o3 = order > 2;
    R h30 = o3 ? h[6] : R(0), h21 = o3 ? h[7] : R(0), h12 = o3 ? h[8] : R(0), h03 = o3 ? h[9] : R(0);
    // B[p][iy] = sum_q h[p][q] He_q(c_iy), p = x degree
    R B0[4], B1[4], B2[4], B3[4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const R c = m ? Lat<R>::cb : Lat<R>::ca;
        const R e2 = m ? Lat<R>::he2b : Lat<R>::he2a;
        const R e3 = m ? Lat<R>::he3b : Lat<R>::he3a;
        const int ip = m ? 3 : 2, im = m ? 0 : 1;
        R E = h[0] + h[5] * e2, O = h[2] * c + h03 * e3;
        B0[ip] = E + O;
        B0[im] = E - O;
        E = h[1] + h12 * e2;
        O = h[4] * c;
        B1[ip] = E + O;
        B1[im] = E - O;
        E = h[3];
        O = h21 * c;
        B2[ip] = E + O;
        B2[im] = E - O;
        B3[ip] = h30;
        B3[im] = h30;
    }
#pragma unroll
    for (int iy = 0; iy < 4; ++iy) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const R c = m ? Lat<R>::cb : Lat<R>::ca;
            const R e2 = m ? Lat<R>::he2b : Lat<R>::he2a;
            const R e3 = m ? Lat<R>::he3b : Lat<R>::he3a;
            const int ip = m ? 3 : 2, im = m ? 0 : 1;
            R E = B0[iy] + B2[iy] * e2, O = B1[iy] * c + B3[iy] * e3;
            p[ip + 4 * iy] = E + O;
            p[im + 4 * iy] = E - O;
        }
    }
}


// 2D reduced populations of the node columns in `cols` only (bit n: normal node n, in
// node order -cb, -ca, +ca, +cb), normal axis AXIS, sum factorization over the normal
// direction first; the populations of the other columns are set to 0. `cols` must be the
// same in every lane of the wave (the column loop branches on it).
template <typename R, int AXIS>
PD void eval_cols_2d(const R h[10], int cols, R p[16], int order)
{
    const bool o3 = order > 2;
    // coefficients as g[n][t]: n = normal degree, t = tangential degree
    R g00 = h[0], g10, g01, g20, g11, g02, g30, g21, g12, g03;
    if (AXIS == 0) {
        g10 = h[1]; g01 = h[2]; g20 = h[3]; g11 = h[4]; g02 = h[5];
        g30 = o3 ? h[6] : R(0); g21 = o3 ? h[7] : R(0); g12 = o3 ? h[8] : R(0); g03 = o3 ? h[9] : R(0);
    } else {
        g10 = h[2]; g01 = h[1]; g20 = h[5]; g11 = h[4]; g02 = h[3];
        g30 = o3 ? h[9] : R(0); g21 = o3 ? h[8] : R(0); g12 = o3 ? h[7] : R(0); g03 = o3 ? h[6] : R(0);
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        R out[4] = {R(0), R(0), R(0), R(0)};
        if (cols & (1 << n)) {
            const R cn = node<R>(n);
            const R e2 = (n == 1 || n == 2) ? Lat<R>::he2a : Lat<R>::he2b;
            const R e3n = (n == 1 || n == 2) ? Lat<R>::he3a : Lat<R>::he3b;
            const R e3 = (n < 2) ? -e3n : e3n; // He3 is odd
            // A_t = sum_n' g[n'][t] He_n'(c_n); explicit fma throughout, so that a column's
            // value does not depend on which other columns are evaluated (which products the
            // compiler could otherwise share between columns and leave unfused)
            const R A0 = fma(e3, g30, fma(e2, g20, fma(cn, g10, g00)));
            const R A1 = fma(e2, g21, fma(cn, g11, g01));
            const R A2 = fma(cn, g12, g02);
            const R A3 = g03;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const R ct = m ? Lat<R>::cb : Lat<R>::ca;
                const R t2 = m ? Lat<R>::he2b : Lat<R>::he2a;
                const R t3 = m ? Lat<R>::he3b : Lat<R>::he3a;
                const R E = fma(A2, t2, A0), O = fma(A3, t3, A1 * ct);
                out[m ? 3 : 2] = E + O;
                out[m ? 0 : 1] = E - O;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) p[AXIS ? (t + 4 * n) : (n + 4 * t)] = out[t];
    }
}

// ---------------------------------------------------------------------------------
// 2D coefficients in scaled form q: the Hermite coefficients h_ab times a! b! (q20 = 2 h20,
// q30 = 6 h30, q21 = 2 h21, ...), which turns the conversions to and from raw moments
// into plain additions; the population evaluation takes the factorials into its constants.
// Index order as for h: 00 10 01 20 11 02 30 21 12 03.
// ---------------------------------------------------------------------------------

template <typename R>
PD void q2mu_2d(const R q[10], R mu[10], int n)
{
    mu[0] = q[0];
    mu[1] = q[1];
    mu[2] = q[2];
    mu[3] = q[0] + q[3];
    mu[4] = q[4];
    mu[5] = q[0] + q[5];
    if (n > 6) {
        mu[6] = fma(R(3), q[1], q[6]);
        mu[7] = q[2] + q[7];
        mu[8] = q[1] + q[8];
        mu[9] = fma(R(3), q[2], q[9]);
    }
}

template <typename R>
PD void mu2q_2d(const R mu[10], R q[10], int n)
{
    q[0] = mu[0];
    q[1] = mu[1];
    q[2] = mu[2];
    q[3] = mu[3] - mu[0];
    q[4] = mu[4];
    q[5] = mu[5] - mu[0];
    if (n > 6) {
        q[6] = fma(R(-3), mu[1], mu[6]);
        q[7] = mu[7] - mu[2];
        q[8] = mu[8] - mu[1];
        q[9] = fma(R(-3), mu[2], mu[9]);
    }
}

// He_2 / 2 and He_3 / 6 at the two node magnitudes
template <typename R>
struct LatQ {
    static constexpr R e2a = R(0.5 * Lat<double>::he2a), e2b = R(0.5 * Lat<double>::he2b);
    static constexpr R e3a = R(Lat<double>::he3a / 6.0), e3b = R(Lat<double>::he3b / 6.0);
};

// reduced populations p_i = f_i / W_i from scaled coefficients (sum factorization over y
// then x, as eval_2d)
template <typename R>
PD void eval_q_2d(const R q[10], R p[16], int order)
{
    const bool o3 = order > 2;
    R q30 = o3 ? q[6] : R(0), q21 = o3 ? q[7] : R(0), q12 = o3 ? q[8] : R(0), q03 = o3 ? q[9] : R(0);
    R B0[4], B1[4], B2[4], B3[4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const R c = m ? Lat<R>::cb : Lat<R>::ca;
        const R e2 = m ? LatQ<R>::e2b : LatQ<R>::e2a;
        const R e3 = m ? LatQ<R>::e3b : LatQ<R>::e3a;
        const int ip = m ? 3 : 2, im = m ? 0 : 1;
        R E = fma(q[5], e2, q[0]), O = fma(q03, e3, q[2] * c);
        B0[ip] = E + O;
        B0[im] = E - O;
        E = fma(q12, e2, q[1]);
        O = q[4] * c;
        B1[ip] = E + O;
        B1[im] = E - O;
        E = q[3];
        O = q21 * c;
        B2[ip] = E + O;
        B2[im] = E - O;
        B3[ip] = q30;
        B3[im] = q30;
    }
#pragma unroll
    for (int iy = 0; iy < 4; ++iy) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const R c = m ? Lat<R>::cb : Lat<R>::ca;
            const R e2 = m ? LatQ<R>::e2b : LatQ<R>::e2a;
            const R e3 = m ? LatQ<R>::e3b : LatQ<R>::e3a;
            const int ip = m ? 3 : 2, im = m ? 0 : 1;
            R E = fma(B2[iy], e2, B0[iy]), O = fma(B3[iy], e3, B1[iy] * c);
            p[ip + 4 * iy] = E + O;
            p[im + 4 * iy] = E - O;
        }
    }
}

// the populations of the node columns in `cols` only, from scaled coefficients (as
// eval_cols_2d; explicit fma throughout, so a column's value does not depend on which
// other columns are evaluated)
template <typename R, int AXIS>
PD void eval_q_cols_2d(const R q[10], int cols, R p[16], int order)
{
    const bool o3 = order > 2;
    // G[n][t] = q of normal degree n, tangential degree t
    R g00 = q[0], g10, g01, g20, g11, g02, g30, g21, g12, g03;
    if (AXIS == 0) {
        g10 = q[1]; g01 = q[2]; g20 = q[3]; g11 = q[4]; g02 = q[5];
        g30 = o3 ? q[6] : R(0); g21 = o3 ? q[7] : R(0); g12 = o3 ? q[8] : R(0); g03 = o3 ? q[9] : R(0);
    } else {
        g10 = q[2]; g01 = q[1]; g20 = q[5]; g11 = q[4]; g02 = q[3];
        g30 = o3 ? q[9] : R(0); g21 = o3 ? q[8] : R(0); g12 = o3 ? q[7] : R(0); g03 = o3 ? q[6] : R(0);
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        R out[4] = {R(0), R(0), R(0), R(0)};
        if (cols & (1 << n)) {
            const R cn = node<R>(n);
            const R e2 = (n == 1 || n == 2) ? LatQ<R>::e2a : LatQ<R>::e2b;
            const R e3n = (n == 1 || n == 2) ? LatQ<R>::e3a : LatQ<R>::e3b;
            const R e3 = (n < 2) ? -e3n : e3n; // He3 is odd
            // A_t (times t!) = sum_n' G[n'][t] He_n'(c_n) / n'!
            const R A0 = fma(e3, g30, fma(e2, g20, fma(cn, g10, g00)));
            const R A1 = fma(e2, g21, fma(cn, g11, g01));
            const R A2 = fma(cn, g12, g02);
            const R A3 = g03;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const R ct = m ? Lat<R>::cb : Lat<R>::ca;
                const R t2 = m ? LatQ<R>::e2b : LatQ<R>::e2a;
                const R t3 = m ? LatQ<R>::e3b : LatQ<R>::e3a;
                const R E = fma(A2, t2, A0), O = fma(A3, t3, A1 * ct);
                out[m ? 3 : 2] = E + O;
                out[m ? 0 : 1] = E - O;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) p[AXIS ? (t + 4 * n) : (n + 4 * t)] = out[t];
    }
}

// ---------------------------------------------------------------------------------
// The alternative regularization of Sec. II.C for f (2D): the moments of degree <= 3 are
// kept and the six others of the D2Q16 moment vector (c_x^a c_y^b, a, b <= 3, a + b >= 4,
// in the frame-relative velocities of the new frame) take the values of the product-form
// equilibrium with the state's density and velocity and the frame's temperature. In the
// scaled form the coefficients ARE the Hermite moments q_ab = sum_i f_i He_a He_b, so with
// d = (q10, q01)/q00 the equilibrium's are q00 d_x^a d_y^b and, writing Dq = q - q_eq for the
// kept ones, the condition on the raw moments fixes the other six:
//   q31 = q_eq31 - 3 Dq11, q13 = q_eq13 - 3 Dq11, q22 = q_eq22 - Dq20 - Dq02,
//   q32 = q_eq32 - 3 Dq12 - Dq30, q23 = q_eq23 - 3 Dq21 - Dq03, q33 = q_eq33 + 9 Dq11
// (from c^2 = He2 + 1 and c^3 = He3 + 3 He1 on each axis).
// Fast order: 31 22 13 32 23 33.
// ---------------------------------------------------------------------------------

template <typename R>
PD void eq_fast_2d(const R q[10], R qf[6])
{
    const R rho = q[0];
    const R ir = R(1) / rho;
    const R dx = q[1] * ir, dy = q[2] * ir;
    const R rx = rho * dx, ry = rho * dy;
    const R e20 = rx * dx, e11 = rx * dy, e02 = ry * dy;
    const R d20 = q[3] - e20, d11 = q[4] - e11, d02 = q[5] - e02;
    const R d30 = q[6] - e20 * dx, d21 = q[7] - e20 * dy, d12 = q[8] - e02 * dx, d03 = q[9] - e02 * dy;
    const R e31 = e20 * dx * dy, e22 = e20 * dy * dy, e13 = e02 * dx * dy;
    qf[0] = fma(R(-3), d11, e31);
    qf[1] = e22 - d20 - d02;
    qf[2] = fma(R(-3), d11, e13);
    qf[3] = fma(R(-3), d12, e31 * dy) - d30;
    qf[4] = fma(R(-3), d21, e13 * dx) - d03;
    qf[5] = fma(R(9), d11, e22 * dx * dy);
}

// reduced populations from the 10 kept and 6 fast scaled coefficients (the full tensor
// product of degrees <= 3 per axis; sum factorization over y then x, as eval_q_2d)
template <typename R>
PD void eval_q16_2d(const R q[10], const R qf[6], R p[16])
{
    // rows of x degree a: (a0, a1, a2, a3)
    const R g[4][4] = {{q[0], q[2], q[5], q[9]},
                       {q[1], q[4], q[8], qf[2]},
                       {q[3], q[7], qf[1], qf[4]},
                       {q[6], qf[0], qf[3], qf[5]}};
    R B[4][4];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const R c = m ? Lat<R>::cb : Lat<R>::ca;
        const R e2 = m ? LatQ<R>::e2b : LatQ<R>::e2a;
        const R e3 = m ? LatQ<R>::e3b : LatQ<R>::e3a;
        const int ip = m ? 3 : 2, im = m ? 0 : 1;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const R E = fma(g[a][2], e2, g[a][0]), O = fma(g[a][3], e3, g[a][1] * c);
            B[a][ip] = E + O;
            B[a][im] = E - O;
        }
    }
#pragma unroll
    for (int iy = 0; iy < 4; ++iy) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const R c = m ? Lat<R>::cb : Lat<R>::ca;
            const R e2 = m ? LatQ<R>::e2b : LatQ<R>::e2a;
            const R e3 = m ? LatQ<R>::e3b : LatQ<R>::e3a;
            const int ip = m ? 3 : 2, im = m ? 0 : 1;
            const R E = fma(B[2][iy], e2, B[0][iy]), O = fma(B[3][iy], e3, B[1][iy] * c);
            p[ip + 4 * iy] = E + O;
            p[im + 4 * iy] = E - O;
        }
    }
}

// the populations of the node columns in `cols` only, from the 16 scaled coefficients (as
// eval_q_cols_2d, explicit fma throughout)
template <typename R, int AXIS>
PD void eval_q16_cols_2d(const R q[10], const R qf[6], int cols, R p[16])
{
    // G[n][t]: normal degree n, tangential degree t
    const R gx[4][4] = {{q[0], q[2], q[5], q[9]},
                        {q[1], q[4], q[8], qf[2]},
                        {q[3], q[7], qf[1], qf[4]},
                        {q[6], qf[0], qf[3], qf[5]}};
    R G[4][4];
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int t = 0; t < 4; ++t) G[n][t] = AXIS ? gx[t][n] : gx[n][t];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        R out[4] = {R(0), R(0), R(0), R(0)};
        if (cols & (1 << n)) {
            const R cn = node<R>(n);
            const R e2 = (n == 1 || n == 2) ? LatQ<R>::e2a : LatQ<R>::e2b;
            const R e3n = (n == 1 || n == 2) ? LatQ<R>::e3a : LatQ<R>::e3b;
            const R e3 = (n < 2) ? -e3n : e3n; // He3 is odd
            R A[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) A[t] = fma(e3, G[3][t], fma(e2, G[2][t], fma(cn, G[1][t], G[0][t])));
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const R ct = m ? Lat<R>::cb : Lat<R>::ca;
                const R t2 = m ? LatQ<R>::e2b : LatQ<R>::e2a;
                const R t3 = m ? LatQ<R>::e3b : LatQ<R>::e3a;
                const R E = fma(A[2], t2, A[0]), O = fma(A[3], t3, A[1] * ct);
                out[m ? 3 : 2] = E + O;
                out[m ? 0 : 1] = E - O;
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) p[AXIS ? (t + 4 * n) : (n + 4 * t)] = out[t];
    }
}

// raw moments mu = sum_i W_i p_i c^k (1D), up to degree n-1
template <typename R>
PD void moments_1d(const R p[4], R mu[4], int n)
{
    R s0a = Lat<R>::wa * (p[2] + p[1]), s0b = Lat<R>::wb * (p[3] + p[0]);
    R s1a = Lat<R>::wa * (p[2] - p[1]), s1b = Lat<R>::wb * (p[3] - p[0]);
    const R ca = Lat<R>::ca, cb = Lat<R>::cb;
    mu[0] = s0a + s0b;
    mu[1] = ca * s1a + cb * s1b;
    mu[2] = ca * ca * s0a + cb * cb * s0b;
    if (n > 3) mu[3] = ca * ca * ca * s1a + cb * cb * cb * s1b;
}

// 2D raw moments up to total degree 3 (n = 10) or 2 (n = 6)
template <typename R>
PD void moments_2d(const R p[16], R mu[10], int n)
{
    // weights times node powers, one product per (node pair, degree)
    constexpr R w0a = Lat<R>::wa, w0b = Lat<R>::wb;
    constexpr R w1a = R(Lat<double>::wa * Lat<double>::ca), w1b = R(Lat<double>::wb * Lat<double>::cb);
    constexpr R w2a = R(Lat<double>::wa * Lat<double>::ca * Lat<double>::ca);
    constexpr R w2b = R(Lat<double>::wb * Lat<double>::cb * Lat<double>::cb);
    constexpr R w3a = R(Lat<double>::wa * Lat<double>::ca * Lat<double>::ca * Lat<double>::ca);
    constexpr R w3b = R(Lat<double>::wb * Lat<double>::cb * Lat<double>::cb * Lat<double>::cb);
    // reduce over y for every column ix: Rl[ix] = sum_iy w_iy c_iy^l p(ix, iy)
    R R0[4], R1[4], R2[4], R3[4];
#pragma unroll
    for (int ix = 0; ix < 4; ++ix) {
        R ea = p[ix + 8] + p[ix + 4], oa = p[ix + 8] - p[ix + 4];
        R eb = p[ix + 12] + p[ix], ob = p[ix + 12] - p[ix];
        R0[ix] = fma(w0b, eb, w0a * ea);
        R1[ix] = fma(w1b, ob, w1a * oa);
        R2[ix] = fma(w2b, eb, w2a * ea);
        R3[ix] = fma(w3b, ob, w3a * oa);
    }
    // reduce over x
    auto red = [&](const R* Rl, R& m0, R& m1, R& m2, R& m3) {
        R ea = Rl[2] + Rl[1], oa = Rl[2] - Rl[1];
        R eb = Rl[3] + Rl[0], ob = Rl[3] - Rl[0];
        m0 = fma(w0b, eb, w0a * ea);
        m1 = fma(w1b, ob, w1a * oa);
        m2 = fma(w2b, eb, w2a * ea);
        m3 = fma(w3b, ob, w3a * oa);
    };
    R a0, a1, a2, a3;
    red(R0, a0, a1, a2, a3);
    mu[0] = a0;
    mu[1] = a1;
    mu[3] = a2;
    if (n > 6) mu[6] = a3;
    red(R1, a0, a1, a2, a3);
    mu[2] = a0;
    mu[4] = a1;
    if (n > 6) mu[7] = a2;
    red(R2, a0, a1, a2, a3);
    mu[5] = a0;
    if (n > 6) mu[8] = a1;
    if (n > 6) {
        red(R3, a0, a1, a2, a3);
        mu[9] = a0;
    }
}

// Moments of the reduced populations in two stages, tangential then normal, so that the
// populations can be produced half a face at a time (two normal node columns): the
// tangential stage of normal node n gives the weighted tangential power sums of degree
// 0..3 of that column's 4 populations (tangential node t at p[t]); the normal stage then
// combines the 4 columns into the moments mu (layout 00 10 01 20 11 02 30 21 12 03 in
// x-y powers; n = 6 for degree 2). For AXIS = 0 this is moments_2d's own order.
template <typename R>
PD void tan_sums(const R p0, const R p1, const R p2, const R p3, R out[4])
{
    constexpr R w0a = Lat<R>::wa, w0b = Lat<R>::wb;
    constexpr R w1a = R(Lat<double>::wa * Lat<double>::ca), w1b = R(Lat<double>::wb * Lat<double>::cb);
    constexpr R w2a = R(Lat<double>::wa * Lat<double>::ca * Lat<double>::ca);
    constexpr R w2b = R(Lat<double>::wb * Lat<double>::cb * Lat<double>::cb);
    constexpr R w3a = R(Lat<double>::wa * Lat<double>::ca * Lat<double>::ca * Lat<double>::ca);
    constexpr R w3b = R(Lat<double>::wb * Lat<double>::cb * Lat<double>::cb * Lat<double>::cb);
    const R ea = p2 + p1, oa = p2 - p1;
    const R eb = p3 + p0, ob = p3 - p0;
    out[0] = fma(w0b, eb, w0a * ea);
    out[1] = fma(w1b, ob, w1a * oa);
    out[2] = fma(w2b, eb, w2a * ea);
    out[3] = fma(w3b, ob, w3a * oa);
}

template <typename R, int AXIS>
PD void normal_sums(const R Rt[4][4], R mu[10], int n)
{
    R m[4][4]; // [tangential degree l][normal degree k]
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        R col[4] = {Rt[0][l], Rt[1][l], Rt[2][l], Rt[3][l]};
        tan_sums(col[0], col[1], col[2], col[3], m[l]);
    }
    // (x degree, y degree) -> index
    auto at = [](int a, int b) {
        const int d = a + b;
        return d * (d + 1) / 2 + b;
    };
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int a = AXIS ? l : k, b = AXIS ? k : l;
            if (a + b <= (n > 6 ? 3 : 2)) mu[at(a, b)] = m[l][k];
        }
}

// reciprocal without the scaling and fix-up of IEEE division: the hardware estimate in FP32
// (1 ulp), and in FP64 the estimate refined by two Newton steps (a few ulp); the limiter
// and the frame update only need this accuracy
PD float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }
PD double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    return r * (2.0 - x * r);
}

// Reciprocal and reciprocal square root of the frame update: in FP32 the hardware estimates
// (about 1 ulp; the FP32 form is not held to bit equality with the FP64 oracle), in FP64 the
// correctly rounded operations.
PD float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
PD double frcp(double x) { return 1.0 / x; }
PD float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
PD double frsq(double x) { return 1.0 / sqrt(x); }

// slope limiters of the MUSCL reconstruction (Van Leer, minmod)
template <typename R>
PD R limit(R a, R b, int kind)
{
    R ab = a * b;
    if (!(ab > R(0))) return R(0);
    if (kind == 1) return (a > R(0)) ? fmin(a, b) : fmax(a, b);
    return R(2) * ab * rcp_nr(a + b);
}

// the limited slope divided by limit_scale(kind): Van Leer without its factor 2, which the
// caller folds into the offset the slope multiplies (a power of two, so the product is
// bitwise that of limit())
template <typename R>
PD R limit_part(R a, R b, int kind)
{
    R ab = a * b;
    if (!(ab > R(0))) return R(0);
    if (kind == 1) return (a > R(0)) ? fmin(a, b) : fmax(a, b);
    return ab * rcp_nr(a + b);
}
PD constexpr int limit_scale(int kind) { return kind == 1 ? 1 : 2; }

} // namespace pond
