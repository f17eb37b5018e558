/*
 * pond_oracle.c -- plain, slow, FP64 CPU oracle of the finite-volume
 * Particles-on-Demand (PonD) time step of Kallikounis, Dorschner & Karlin,
 * "Particles on Demand for flows with strong discontinuities".
 *
 * TEST INFRASTRUCTURE. This is the reference the HIP library is checked against.
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it. It shares no code, header, table or constant with the GPU library.
 *
 * The step follows the paper's own summary of the finite-volume algorithm
 * (Sec. III.B.4): a loop over cells that expresses every cell's populations in
 * its co-moving frame, a loop over cells that forms phi-bar-plus, a loop over
 * faces that runs the predictor-corrector frame iteration of Sec. III.B.3, and a
 * loop over cells that converts the face fluxes into each cell's frame and applies
 * the co-moving update of Sec. III.B.2. All arithmetic is IEEE double precision
 * (no fast-math), written with explicit loops and full tensors in the paper's
 * lab-frame notation (moments M_k, Grad coefficients a_k).
 *
 * Readings where the paper is silent (each repeated where it is used):
 *  - gas constant R = 1, so p = rho T and C_v = 1/(gamma-1);
 *  - tau = mu/p (Chapman-Enskog for single-relaxation BGK, Prandtl 1), and every
 *    relaxation coefficient is written with eps = dt/tau = dt p/mu;
 *  - the "overline" symmetrization of Sec. II.C sums the distinct index
 *    permutations without a 1/n! factor;
 *  - Van Leer limiter by default, minmod on request, zero on a sign change or zero;
 *  - upwind cell is the left/lower one when the normal component v_i.n >= 0;
 *  - frame convergence: max(|u^(k+1)-u^(k)|_inf / sqrt(T^(k+1)),
 *    |T^(k+1)-T^(k)| / T^(k+1)) <= tol; the face keeps the moments of the last
 *    reconstruction and the frame computed from them; an iteration that returns to
 *    within 1e-2 of its last step of the frame two iterations back (a 2-cycle, which
 *    the discontinuous upwind choice can produce) stops there as non-converged, as
 *    does one that reaches max_iter;
 *  - seed of the first step: frame of the mean conserved variables of the two
 *    cells next to the face; later steps: the face frame of the previous step;
 *  - the face equilibrium used to recover phi from phi-bar is the co-moving
 *    equilibrium of the face's final frame, applied to the moments;
 *  - the time step: CFL = max |v_ia| dt/dx_a over the populations of every cell and of
 *    every state a boundary condition prescribes (they enter through boundary faces),
 *    recomputed every step from the cell frames at its start;
 *  - two ghost layers; x-ghosts are filled for the interior rows first, then the
 *    y-ghosts of every column (so corner ghosts take the y rule of an x-ghost);
 *  - a corrector frame with rho <= 0 or T <= 0 restarts the iteration once from
 *    the frame of the mean conserved variables of the two neighbours; a second
 *    such frame, or an iteration that stops without converging, switches the face to
 *    the first-order upwind state assembled from each neighbour's populations in that
 *    neighbour's own frame.
 */
#include "pond_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TL 1.0 /* lattice temperature of Table I */
#define MAXD 3
#define MAXQ 64
#define NG 2 /* ghost layers */

/* ------------------------------------------------------------------------- */
/* lattice (Sec. II.A, Table I)                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    int D, Q;
    double c[MAXQ][MAXD];
    double W[MAXQ];
} lattice;

/* D1Q4 nodes are the roots of the fourth Hermite polynomial, +-sqrt(3 -+ sqrt 6),
 * with Gauss-Hermite weights (3 +- sqrt 6)/12; D2Q16 is their tensor product,
 * W_i = w_ix w_iy, and D3Q64 the product of three. Index i = ix + 4 iy + 16 iz with nodes
 * sorted ascending. */
static void make_lattice(int D, lattice *L)
{
    const double r6 = sqrt(6.0);
    const double c1[4] = {-sqrt(3.0 + r6), -sqrt(3.0 - r6), sqrt(3.0 - r6), sqrt(3.0 + r6)};
    const double w1[4] = {(3.0 - r6) / 12.0, (3.0 + r6) / 12.0, (3.0 + r6) / 12.0,
                          (3.0 - r6) / 12.0};
    memset(L, 0, sizeof(*L));
    L->D = D;
    L->Q = (D == 1) ? 4 : (D == 2) ? 16 : 64;
    for (int i = 0; i < L->Q; ++i) {
        int ix = i % 4, iy = (i / 4) % 4, iz = i / 16;
        L->c[i][0] = c1[ix];
        L->W[i] = w1[ix];
        if (D >= 2) {
            L->c[i][1] = c1[iy];
            L->W[i] *= w1[iy];
        }
        if (D == 3) {
            L->c[i][2] = c1[iz];
            L->W[i] *= w1[iz];
        }
    }
}

int orc_lattice(int dim, double *c, double *W)
{
    lattice L;
    make_lattice(dim, &L);
    for (int i = 0; i < L.Q; ++i) {
        for (int a = 0; a < dim; ++a) c[i * dim + a] = L.c[i][a];
        W[i] = L.W[i];
    }
    return L.Q;
}

/* particle velocities in frame lambda = {u, T}: v_i = sqrt(T/T_L) c_i + u (Sec. II.C) */
static void velocities(const lattice *L, const double *u, double T, double v[MAXQ][MAXD])
{
    double s = sqrt(T / TL);
    for (int i = 0; i < L->Q; ++i)
        for (int a = 0; a < L->D; ++a) v[i][a] = s * L->c[i][a] + u[a];
}

/* ------------------------------------------------------------------------- */
/* moment tensors and the Grad projection (Sec. II.C)                        */
/* ------------------------------------------------------------------------- */

typedef struct {
    double t0;
    double t1[MAXD];
    double t2[MAXD][MAXD];
    double t3[MAXD][MAXD][MAXD];
} tensors;

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* M_k = sum_i f_i v_i (x) ... (x) v_i, k = 0..3, in the lab frame */
static void moments(const lattice *L, const double *f, const double *u, double T, tensors *M)
{
    double v[MAXQ][MAXD];
    const int D = L->D;
    velocities(L, u, T, v);
    memset(M, 0, sizeof(*M));
    for (int i = 0; i < L->Q; ++i) {
        M->t0 += f[i];
        for (int a = 0; a < D; ++a) {
            M->t1[a] += f[i] * v[i][a];
            for (int b = 0; b < D; ++b) {
                M->t2[a][b] += f[i] * v[i][a] * v[i][b];
                for (int c = 0; c < D; ++c) M->t3[a][b][c] += f[i] * v[i][a] * v[i][b] * v[i][c];
            }
        }
    }
}

/* Grad coefficients that make the projected populations reproduce M_0..M_order in
 * the target frame {u', T'}: the closed forms for a_0, a_1, a_2, a_3 of Sec. II.C
 * (with T_L = 1 kept explicit). */
static void grad_coefficients(int D, int order, const tensors *M, const double *up, double Tp,
                              tensors *a)
{
    const double th = Tp / TL;
    const double sq = sqrt(th);
    memset(a, 0, sizeof(*a));
    a->t0 = M->t0;
    for (int al = 0; al < D; ++al) a->t1[al] = (M->t1[al] - M->t0 * up[al]) / sq;
    for (int al = 0; al < D; ++al)
        for (int be = 0; be < D; ++be) {
            double sym_u_a1 = up[al] * a->t1[be] + up[be] * a->t1[al];
            a->t2[al][be] = (M->t2[al][be] - M->t0 * Tp * kd(al, be) - sq * sym_u_a1 -
                             M->t0 * up[al] * up[be]) /
                            th;
        }
    if (order < 3) return;
    for (int al = 0; al < D; ++al)
        for (int be = 0; be < D; ++be)
            for (int ga = 0; ga < D; ++ga) {
                /* sym(u' (x) (M0 T_L I + a2)) */
                double s1 = up[al] * (M->t0 * TL * kd(be, ga) + a->t2[be][ga]) +
                            up[be] * (M->t0 * TL * kd(al, ga) + a->t2[al][ga]) +
                            up[ga] * (M->t0 * TL * kd(al, be) + a->t2[al][be]);
                /* sym(a1 (x) I) */
                double s2 = a->t1[al] * kd(be, ga) + a->t1[be] * kd(al, ga) + a->t1[ga] * kd(al, be);
                /* sym(a1 (x) u' (x) u') */
                double s3 = a->t1[al] * up[be] * up[ga] + a->t1[be] * up[al] * up[ga] +
                            a->t1[ga] * up[al] * up[be];
                a->t3[al][be][ga] = (M->t3[al][be][ga] - th * s1 - Tp * sq * s2 - sq * s3 -
                                     M->t0 * up[al] * up[be] * up[ga]) /
                                    (th * sq);
            }
}

/* the Grad expansion of Sec. II.C: f_i = W_i (a0 + a1.c/T_L + a2:(cc - T_L I)/(2 T_L^2)
 * + a3:(ccc - T_L sym(c (x) I))/(6 T_L^3)); order 2 drops the last term */
static void grad_populations(const lattice *L, int order, const tensors *a, double *f)
{
    const int D = L->D;
    for (int i = 0; i < L->Q; ++i) {
        const double *c = L->c[i];
        double s = a->t0;
        for (int al = 0; al < D; ++al) s += a->t1[al] * c[al] / TL;
        for (int al = 0; al < D; ++al)
            for (int be = 0; be < D; ++be)
                s += a->t2[al][be] * (c[al] * c[be] - TL * kd(al, be)) / (2.0 * TL * TL);
        if (order >= 3)
            for (int al = 0; al < D; ++al)
                for (int be = 0; be < D; ++be)
                    for (int ga = 0; ga < D; ++ga) {
                        double h3 = c[al] * c[be] * c[ga] -
                                    TL * (c[al] * kd(be, ga) + c[be] * kd(al, ga) + c[ga] * kd(al, be));
                        s += a->t3[al][be][ga] * h3 / (6.0 * TL * TL * TL);
                    }
        f[i] = L->W[i] * s;
    }
}

static void grad_project(const lattice *L, int order, const tensors *M, const double *up,
                         double Tp, double *f)
{
    tensors a;
    grad_coefficients(L->D, order, M, up, Tp, &a);
    grad_populations(L, order, &a, f);
}

/* The alternative regularization of Sec. II.C: in the new frame the moments of order
 * 0..3 keep their values, the remaining Q - q moments take their equilibrium values, and
 * the populations follow from the Q x Q moment system of the new frame.
 * Readings (the paper leaves both open):
 *  - the moment vector is that of the frame-relative velocities c = (v - u')/sqrt(T'),
 *    the monomials c_x^a c_y^b with 0 <= a, b <= 3 (independent on the product lattice);
 *    the slow ones are a + b <= 3 (they carry the same information as M_0..M_3), the fast
 *    ones a + b >= 4. Monomials of the lab velocities would make the result depend on
 *    the lab velocity of the frame itself (not Galilean invariant), which the frame-relative
 *    ones do not;
 *  - the equilibrium of the fast moments depends on M_0 and M_1 only: it is the
 *    product-form equilibrium of the new frame's lattice with density M_0 and velocity
 *    M_1/M_0, i.e. in frame-relative variables rho g_a(d_x) g_b(d_y) with
 *    d = (M_1/M_0 - u')/sqrt(T') and the unit-variance Gaussian moments
 *    g_0 = 1, g_1 = d, g_2 = d^2 + 1, g_3 = d^3 + 3 d.
 * D1Q4 has Q = q: no fast moments, the Grad projection is the same transformation. */
static double ipow(double x, int n)
{
    double r = 1.0;
    for (int k = 0; k < n; ++k) r *= x;
    return r;
}

static double binom(int n, int k)
{
    double r = 1.0;
    for (int j = 1; j <= k; ++j) r = r * (n - k + j) / j;
    return r;
}

/* lab moment with a x-components and b y-components, a + b <= 3 */
static double lab_moment(const tensors *M, int a, int b)
{
    int idx[3], n = 0;
    for (int k = 0; k < a; ++k) idx[n++] = 0;
    for (int k = 0; k < b; ++k) idx[n++] = 1;
    if (n == 0) return M->t0;
    if (n == 1) return M->t1[idx[0]];
    if (n == 2) return M->t2[idx[0]][idx[1]];
    return M->t3[idx[0]][idx[1]][idx[2]];
}

/* solve A x = b (n x n, row-major in A[n][n+1] with b as the last column) by Gaussian
 * elimination with partial pivoting */
static void gauss_solve(int n, double A[MAXQ][MAXQ + 1], double *x)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col)
            for (int k = 0; k <= n; ++k) {
                double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
        for (int r = col + 1; r < n; ++r) {
            double m = A[r][col] / A[col][col];
            for (int k = col; k <= n; ++k) A[r][k] -= m * A[col][k];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double acc = A[r][n];
        for (int k = r + 1; k < n; ++k) acc -= A[r][k] * x[k];
        x[r] = acc / A[r][r];
    }
}

static void eq_project(const lattice *L, const tensors *M, const double *up, double Tp, double *f)
{
    if (L->D == 1) {
        grad_project(L, 3, M, up, Tp, f);
        return;
    }
    const double s = sqrt(Tp / TL);
    const double rho = M->t0;
    const double d[2] = {(M->t1[0] / rho - up[0]) / s, (M->t1[1] / rho - up[1]) / s};
    double g[2][4];
    for (int a = 0; a < 2; ++a) {
        g[a][0] = 1.0;
        g[a][1] = d[a];
        g[a][2] = d[a] * d[a] + 1.0;
        g[a][3] = d[a] * d[a] * d[a] + 3.0 * d[a];
    }
    double A[MAXQ][MAXQ + 1];
    int row = 0;
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a, ++row) {
            for (int i = 0; i < L->Q; ++i) A[row][i] = ipow(L->c[i][0], a) * ipow(L->c[i][1], b);
            double rhs = 0.0;
            if (a + b <= 3) {
                /* frame-relative moment from the lab ones: expand
                 * ((v_x - u'_x)/s)^a ((v_y - u'_y)/s)^b binomially */
                for (int k = 0; k <= a; ++k)
                    for (int l = 0; l <= b; ++l)
                        rhs += binom(a, k) * binom(b, l) * ipow(-up[0], a - k) * ipow(-up[1], b - l) *
                               lab_moment(M, k, l);
                rhs /= ipow(s, a + b);
            } else {
                rhs = rho * g[0][a] * g[1][b];
            }
            A[row][L->Q] = rhs;
        }
    gauss_solve(L->Q, A, f);
}

/* the f-population transformation of the configured regularization */
static void project_f(const lattice *L, int reg, const tensors *M, const double *up, double Tp, double *f)
{
    if (reg == ORC_REG_EQ)
        eq_project(L, M, up, Tp, f);
    else
        grad_project(L, 3, M, up, Tp, f);
}

/* packing helpers for the exported unit functions */
static void pack(int D, int order, const tensors *M, double *out)
{
    int k = 0;
    out[k++] = M->t0;
    if (order >= 1)
        for (int a = 0; a < D; ++a) out[k++] = M->t1[a];
    if (order >= 2)
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) out[k++] = M->t2[a][b];
    if (order >= 3)
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                for (int c = 0; c < D; ++c) out[k++] = M->t3[a][b][c];
}

static void unpack(int D, int order, const double *in, tensors *M)
{
    int k = 0;
    memset(M, 0, sizeof(*M));
    M->t0 = in[k++];
    if (order >= 1)
        for (int a = 0; a < D; ++a) M->t1[a] = in[k++];
    if (order >= 2)
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) M->t2[a][b] = in[k++];
    if (order >= 3)
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b)
                for (int c = 0; c < D; ++c) M->t3[a][b][c] = in[k++];
}

void orc_moments(int dim, int order, const double *f, const double *u, double T, double *M)
{
    lattice L;
    tensors t;
    make_lattice(dim, &L);
    moments(&L, f, u, T, &t);
    pack(dim, order, &t, M);
}

void orc_grad_project(int dim, int order, const double *M, const double *u, double T, double *f)
{
    lattice L;
    tensors t;
    make_lattice(dim, &L);
    unpack(dim, order, M, &t);
    grad_project(&L, order, &t, u, T, f);
}

void orc_eq_project(int dim, const double *M, const double *u, double T, double *f)
{
    lattice L;
    tensors t;
    make_lattice(dim, &L);
    unpack(dim, 3, M, &t);
    eq_project(&L, &t, u, T, f);
}

void orc_grad_coefficients(int dim, int order, const double *M, const double *u, double T, double *a)
{
    tensors t, c;
    unpack(dim, order, M, &t);
    grad_coefficients(dim, order, &t, u, T, &c);
    pack(dim, order, &c, a);
}

/* ------------------------------------------------------------------------- */
/* relaxation maps (Sec. III.B.1-3), all in terms of eps = dt/tau            */
/* ------------------------------------------------------------------------- */

/* phi from the carried variable phi~ = phi - (dt/2tau)(phi_eq - phi) */
static double phi_from_tilde(double ft, double feq, double eps)
{
    return (2.0 * ft + eps * feq) / (2.0 + eps);
}

/* phi-bar-plus = phi + (h/2)(phi_eq - phi)/tau with h = dt/2, i.e. + (eps/4)(phi_eq - phi) */
double orc_phibar_plus(double ftilde, double feq, double eps)
{
    double phi = phi_from_tilde(ftilde, feq, eps);
    return phi + 0.25 * eps * (feq - phi);
}

/* phi at the face from phi-bar = phi - (eps/4)(phi_eq - phi), eps = dt/tau at the face */
double orc_face_recover(double phibar, double feq, double eps_face)
{
    return (phibar + 0.25 * eps_face * feq) / (1.0 + 0.25 * eps_face);
}

/* collision part of the co-moving update: ((2tau-dt)/(2tau+dt)) phi~ + (2dt/(2tau+dt)) phi_eq */
double orc_update_relax(double ftilde, double feq, double eps)
{
    return ((2.0 - eps) / (2.0 + eps)) * ftilde + (2.0 * eps / (2.0 + eps)) * feq;
}

/* slope limiters: backward and forward one-sided differences */
double orc_limiter(int kind, double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    if (kind == ORC_LIM_MINMOD) return (a > 0.0) ? fmin(a, b) : fmax(a, b);
    return 2.0 * a * b / (a + b); /* Van Leer */
}

/* ------------------------------------------------------------------------- */
/* simulation state                                                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    double f[MAXQ], g[MAXQ]; /* populations (carried f~, g~; or phi-bar-plus for stencils) */
    double u[MAXD], T;       /* frame the populations are expressed in */
    double rho;              /* density of the cell (zeroth moment)    */
} cellrec;

typedef struct {
    double Mf[1 + MAXD + MAXD * MAXD + MAXD * MAXD * MAXD];
    double Mg[1 + MAXD + MAXD * MAXD];
    double u[MAXD], T;   /* final face frame (seed of the next step) */
    double su[MAXD], sT; /* seed                                     */
    int seeded;
    int iters;
} facerec;

struct orc_sim {
    orc_config cfg;
    lattice L;
    int D, Q, nx, ny, nz, nxg, nyg, nzg;
    double dx[MAXD];
    double Cv;
    double t;
    long long nstep;
    cellrec *cell;   /* carried state, interior + ghost storage (ghosts unused) */
    cellrec *plus;   /* phi-bar-plus of every cell, ghosts included             */
    facerec *face;   /* x-faces, then y-faces, then z-faces                     */
    long long nfx, nfy, nfz;
};

static inline long long cidx3(const orc_sim *s, int i, int j, int k)
{
    return (long long)(i + NG) + (long long)s->nxg * (long long)(s->D >= 2 ? (j + NG) : 0) +
           (long long)s->nxg * s->nyg * (long long)(s->D == 3 ? (k + NG) : 0);
}

static inline long long cidx(const orc_sim *s, int i, int j) { return cidx3(s, i, j, 0); }

static double xc(const orc_sim *s, int i) { return s->cfg.x0 + (i + 0.5) * s->dx[0]; }
static double yc(const orc_sim *s, int j) { return s->D >= 2 ? s->cfg.y0 + (j + 0.5) * s->dx[1] : 0.0; }

/* equilibrium populations of Sec. II.B in the co-moving frame {u, T}:
 * f_eq = rho W_i, g_eq = (C_v - D/2) T rho W_i */
static void set_equilibrium(const orc_sim *s, cellrec *c, double rho, const double *u, double T)
{
    for (int i = 0; i < s->Q; ++i) {
        c->f[i] = rho * s->L.W[i];
        c->g[i] = (s->Cv - 0.5 * s->D) * T * rho * s->L.W[i];
    }
    for (int a = 0; a < s->D; ++a) c->u[a] = u[a];
    c->T = T;
    c->rho = rho;
}

static void set_equilibrium_prim(const orc_sim *s, cellrec *c, const double *st /* rho ux uy p */)
{
    double u[MAXD] = {st[1], st[2], 0.0};
    set_equilibrium(s, c, st[0], u, st[3] / st[0]);
}

/* rho, u, T of populations f, g held in frame (u, T): Sec. II.B definitions
 * rho = sum f, rho u = sum v f, rho E = sum v^2/2 f + sum g, rho E = C_v rho T + rho u^2/2 */
static void macro(const orc_sim *s, const double *f, const double *g, const double *u, double T,
                  double *rho, double *uo, double *To)
{
    tensors Mf, Mg;
    moments(&s->L, f, u, T, &Mf);
    moments(&s->L, g, u, T, &Mg);
    double r = Mf.t0;
    double ke = 0.0, tr = 0.0;
    for (int a = 0; a < s->D; ++a) {
        uo[a] = Mf.t1[a] / r;
        ke += uo[a] * uo[a];
        tr += Mf.t2[a][a];
    }
    double rhoE = 0.5 * tr + Mg.t0;
    *rho = r;
    *To = (rhoE / r - 0.5 * ke) / s->Cv;
}

/* express a cell's populations in its own co-moving frame (Sec. III.B.4, first loop):
 * third-order Grad projection for f, second order for g (Sec. II.C) */
static void reframe_cell(const orc_sim *s, const cellrec *in, cellrec *out)
{
    tensors Mf, Mg;
    double rho, u[MAXD] = {0, 0}, T;
    macro(s, in->f, in->g, in->u, in->T, &rho, u, &T);
    moments(&s->L, in->f, in->u, in->T, &Mf);
    moments(&s->L, in->g, in->u, in->T, &Mg);
    project_f(&s->L, s->cfg.reg, &Mf, u, T, out->f);
    grad_project(&s->L, 2, &Mg, u, T, out->g);
    for (int a = 0; a < s->D; ++a) out->u[a] = u[a];
    out->T = T;
    out->rho = rho;
}

orc_sim *orc_create3(const orc_config *cfg, const double *rho, const double *ux, const double *uy,
                     const double *uz, const double *p)
{
    if (!cfg || cfg->dim < 1 || cfg->dim > 3 || cfg->nx < 2) return NULL;
    if (cfg->dim >= 2 && cfg->ny < 2) return NULL;
    if (cfg->dim == 3 && cfg->nz < 2) return NULL;
    if (!(cfg->gamma > 1.0)) return NULL;
    if (cfg->dim == 3) {
        /* 3D: Grad projection, finite volumes, and the periodic / outflow / reflecting sides */
        if (cfg->reg != ORC_REG_GRAD || cfg->scheme != ORC_SCHEME_FV) return NULL;
        for (int q = 0; q < 6; ++q) {
            int kind = q < 4 ? cfg->bc[q] : cfg->bc_z[q - 4];
            if (kind != ORC_BC_PERIODIC && kind != ORC_BC_OUTFLOW && kind != ORC_BC_REFLECT) return NULL;
        }
    }
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->cfg = *cfg;
    s->D = cfg->dim;
    make_lattice(s->D, &s->L);
    s->Q = s->L.Q;
    s->nx = cfg->nx;
    s->ny = (s->D >= 2) ? cfg->ny : 1;
    s->nz = (s->D == 3) ? cfg->nz : 1;
    s->nxg = s->nx + 2 * NG;
    s->nyg = (s->D >= 2) ? s->ny + 2 * NG : 1;
    s->nzg = (s->D == 3) ? s->nz + 2 * NG : 1;
    s->dx[0] = (cfg->x1 - cfg->x0) / s->nx;
    s->dx[1] = (s->D >= 2) ? (cfg->y1 - cfg->y0) / s->ny : 1.0;
    s->dx[2] = (s->D == 3) ? (cfg->z1 - cfg->z0) / s->nz : 1.0;
    s->Cv = 1.0 / (cfg->gamma - 1.0);
    long long ncg = (long long)s->nxg * s->nyg * s->nzg;
    s->cell = (cellrec *)calloc((size_t)ncg, sizeof(cellrec));
    s->plus = (cellrec *)calloc((size_t)ncg, sizeof(cellrec));
    s->nfx = (long long)(s->nx + 1) * s->ny * s->nz;
    s->nfy = (s->D >= 2) ? (long long)s->nx * (s->ny + 1) * s->nz : 0;
    s->nfz = (s->D == 3) ? (long long)s->nx * s->ny * (s->nz + 1) : 0;
    s->face = (facerec *)calloc((size_t)(s->nfx + s->nfy + s->nfz), sizeof(facerec));
    /* initial state: local equilibrium in the co-moving frame, so f~ = f = f_eq */
    for (int kz = 0; kz < s->nz; ++kz)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                long long k = (long long)i + (long long)s->nx * (j + (long long)s->ny * kz);
                double u[MAXD] = {ux[k], (s->D >= 2 && uy) ? uy[k] : 0.0, (s->D == 3 && uz) ? uz[k] : 0.0};
                if (!(rho[k] > 0.0) || !(p[k] > 0.0)) {
                    orc_destroy(s);
                    return NULL;
                }
                set_equilibrium(s, &s->cell[cidx3(s, i, j, kz)], rho[k], u, p[k] / rho[k]);
            }
    return s;
}

orc_sim *orc_create(const orc_config *cfg, const double *rho, const double *ux, const double *uy,
                    const double *p)
{
    if (cfg && cfg->dim == 3) return NULL; /* 3D needs the z velocity: orc_create3 */
    return orc_create3(cfg, rho, ux, uy, NULL, p);
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->cell);
    free(s->plus);
    free(s->face);
    free(s);
}

double orc_time(const orc_sim *s) { return s->t; }
long long orc_steps(const orc_sim *s) { return s->nstep; }
long long orc_nfaces(const orc_sim *s) { return s->nfx + s->nfy + s->nfz; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* boundary ghosts (applied to the phi-bar-plus records)                     */
/* ------------------------------------------------------------------------- */

/* mirror a record across an axis: population of node c_i goes to the node with the
 * opposite component along that axis, and the frame velocity component flips */
static void mirror(const orc_sim *s, const cellrec *in, cellrec *out, int axis)
{
    *out = *in;
    for (int i = 0; i < s->Q; ++i) {
        int dig[3] = {i % 4, (i / 4) % 4, i / 16};
        dig[axis] = 3 - dig[axis];
        int im = dig[0] + 4 * dig[1] + 16 * dig[2];
        out->f[im] = in->f[i];
        out->g[im] = in->g[i];
    }
    out->u[axis] = -in->u[axis];
}

/* ghost rule of one side. side: 0 W, 1 E, 2 S, 3 N. (gi, gj) ghost index;
 * interior neighbour along the normal is taken from `plus` (already filled). */
static void fill_ghost(orc_sim *s, int side, int gi, int gj)
{
    const int axis = side / 2;
    const int n = (axis == 0) ? s->nx : s->ny;
    int g = (axis == 0) ? gi : gj;        /* ghost coordinate along the normal */
    int layer = (g < 0) ? (-1 - g) : (g - n); /* 0 for the first ghost layer    */
    int kind = s->cfg.bc[side];
    double tpos = (axis == 0) ? yc(s, gj) : xc(s, gi); /* tangential centre */
    cellrec *dst = &s->plus[cidx(s, gi, gj)];
    if (kind == ORC_BC_SPLIT_FIXED_REFLECT)
        kind = (tpos < s->cfg.bc_param[side][0]) ? ORC_BC_FIXED : ORC_BC_REFLECT;
    if (kind == ORC_BC_PERIODIC) {
        int src = (g < 0) ? g + n : g - n;
        *dst = (axis == 0) ? s->plus[cidx(s, src, gj)] : s->plus[cidx(s, gi, src)];
    } else if (kind == ORC_BC_OUTFLOW) {
        int src = (g < 0) ? 0 : n - 1;
        *dst = (axis == 0) ? s->plus[cidx(s, src, gj)] : s->plus[cidx(s, gi, src)];
    } else if (kind == ORC_BC_REFLECT) {
        int src = (g < 0) ? layer : n - 1 - layer;
        const cellrec *in = (axis == 0) ? &s->plus[cidx(s, src, gj)] : &s->plus[cidx(s, gi, src)];
        mirror(s, in, dst, axis);
    } else if (kind == ORC_BC_FIXED) {
        set_equilibrium_prim(s, dst, s->cfg.bc_state[side]);
    } else if (kind == ORC_BC_FIXED_WINDOW) {
        const double *p = s->cfg.bc_param[side];
        set_equilibrium_prim(s, dst, (tpos >= p[0] && tpos <= p[1]) ? s->cfg.bc_alt[side]
                                                                   : s->cfg.bc_state[side]);
    } else if (kind == ORC_BC_MOVING_SHOCK) {
        const double *p = s->cfg.bc_param[side];
        double xs = p[0] + p[1] * (yc(s, gj) + p[2] * s->t);
        set_equilibrium_prim(s, dst, (xc(s, gi) < xs) ? s->cfg.bc_state[side] : s->cfg.bc_alt[side]);
    }
}

/* 3D ghosts (periodic, outflow, reflecting sides): x-ghosts of the interior (y, z) rows,
 * then y-ghosts over every x (ghosts included) of the interior z layers, then z-ghosts over
 * every x and y; side 2a is the lower side of axis a, 2a + 1 the upper */
static void fill_ghost3(orc_sim *s, int axis, int hi, int gi, int gj, int gk)
{
    const int n = axis == 0 ? s->nx : axis == 1 ? s->ny : s->nz;
    int g[3] = {gi, gj, gk};
    int layer = hi ? g[axis] - n : -1 - g[axis];
    int kind = axis < 2 ? s->cfg.bc[2 * axis + hi] : s->cfg.bc_z[hi];
    int src[3] = {gi, gj, gk};
    cellrec *dst = &s->plus[cidx3(s, gi, gj, gk)];
    if (kind == ORC_BC_PERIODIC) {
        src[axis] = hi ? g[axis] - n : g[axis] + n;
        *dst = s->plus[cidx3(s, src[0], src[1], src[2])];
    } else if (kind == ORC_BC_OUTFLOW) {
        src[axis] = hi ? n - 1 : 0;
        *dst = s->plus[cidx3(s, src[0], src[1], src[2])];
    } else { /* reflect */
        src[axis] = hi ? n - 1 - layer : layer;
        mirror(s, &s->plus[cidx3(s, src[0], src[1], src[2])], dst, axis);
    }
}

static void fill_ghosts3(orc_sim *s)
{
    for (int k = 0; k < s->nz; ++k)
        for (int j = 0; j < s->ny; ++j)
            for (int l = 0; l < NG; ++l) {
                fill_ghost3(s, 0, 0, -1 - l, j, k);
                fill_ghost3(s, 0, 1, s->nx + l, j, k);
            }
    for (int k = 0; k < s->nz; ++k)
        for (int i = -NG; i < s->nx + NG; ++i)
            for (int l = 0; l < NG; ++l) {
                fill_ghost3(s, 1, 0, i, -1 - l, k);
                fill_ghost3(s, 1, 1, i, s->ny + l, k);
            }
    for (int j = -NG; j < s->ny + NG; ++j)
        for (int i = -NG; i < s->nx + NG; ++i)
            for (int l = 0; l < NG; ++l) {
                fill_ghost3(s, 2, 0, i, j, -1 - l);
                fill_ghost3(s, 2, 1, i, j, s->nz + l);
            }
}

static void fill_ghosts(orc_sim *s)
{
    if (s->D == 3) {
        fill_ghosts3(s);
        return;
    }
    for (int j = 0; j < s->ny; ++j)
        for (int l = 0; l < NG; ++l) {
            fill_ghost(s, 0, -1 - l, j);
            fill_ghost(s, 1, s->nx + l, j);
        }
    if (s->D == 2)
        for (int i = -NG; i < s->nx + NG; ++i)
            for (int l = 0; l < NG; ++l) {
                fill_ghost(s, 2, i, -1 - l);
                fill_ghost(s, 3, i, s->ny + l);
            }
}

/* ------------------------------------------------------------------------- */
/* the face predictor-corrector (Sec. III.B.3)                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    double dt;
    long long iters_total, nonconv, depout;
    int iters_max;
} stepacc;

/* one face along `axis` between cells L=(iL,jL) and R = L + e_axis */
static void face_iteration(orc_sim *s, facerec *F, int axis, int iL, int jL, int kL, double dt,
                           long long *depout, long long *nonphys)
{
    const int D = s->D, Q = s->Q;
    /* the tangential axes (one in 2D, two in 3D), in increasing order */
    int t_axes[2], nt = 0;
    for (int a = 0; a < D; ++a)
        if (a != axis) t_axes[nt++] = a;
    const double h = 0.5 * dt;
    /* stencil: 0 = L - e_a, 1 = L, 2 = R, 3 = R + e_a; per tangential axis t (q-th):
     * 4 + 4q = L - e_t, 5 + 4q = L + e_t, 6 + 4q = R - e_t, 7 + 4q = R + e_t */
    const int ns = 4 + 4 * nt;
    int sc[12][3];
    const int L0[3] = {iL, jL, kL};
    for (int k = 0; k < ns; ++k)
        for (int a = 0; a < 3; ++a) sc[k][a] = L0[a];
    sc[0][axis] -= 1;
    sc[2][axis] += 1;
    sc[3][axis] += 2;
    for (int q = 0; q < nt; ++q) {
        const int t = t_axes[q], b = 4 + 4 * q;
        sc[b][t] -= 1;
        sc[b + 1][t] += 1;
        sc[b + 2][axis] += 1;
        sc[b + 2][t] -= 1;
        sc[b + 3][axis] += 1;
        sc[b + 3][t] += 1;
    }
    /* lab moments of every stencil cell's phi-bar-plus: they do not depend on the
     * target frame, so the regularized transformation into any lambda is a Grad
     * projection of these (Sec. II.C) */
    tensors Mf[12], Mg[12];
    for (int k = 0; k < ns; ++k) {
        const cellrec *c = &s->plus[cidx3(s, sc[k][0], sc[k][1], sc[k][2])];
        moments(&s->L, c->f, c->u, c->T, &Mf[k]);
        moments(&s->L, c->g, c->u, c->T, &Mg[k]);
    }
    const cellrec *cL = &s->plus[cidx3(s, sc[1][0], sc[1][1], sc[1][2])];
    const cellrec *cR = &s->plus[cidx3(s, sc[2][0], sc[2][1], sc[2][2])];

    /* frame of the mean conserved variables of L and R: the seed of the first step and
     * the restart frame of an iteration that has left the physical states */
    double mu_[MAXD] = {0, 0}, mT;
    {
        double r = 0.5 * (cL->rho + cR->rho), m[MAXD] = {0, 0}, e = 0.0, ke = 0.0;
        const cellrec *cc[2] = {cL, cR};
        for (int q = 0; q < 2; ++q) {
            double u2 = 0.0;
            for (int a = 0; a < D; ++a) {
                m[a] += 0.5 * cc[q]->rho * cc[q]->u[a];
                u2 += cc[q]->u[a] * cc[q]->u[a];
            }
            e += 0.5 * (s->Cv * cc[q]->rho * cc[q]->T + 0.5 * cc[q]->rho * u2);
        }
        for (int a = 0; a < D; ++a) {
            mu_[a] = m[a] / r;
            ke += mu_[a] * mu_[a];
        }
        mT = (e / r - 0.5 * ke) / s->Cv;
    }
    /* predictor frame lambda_0: the face frame of the previous half step */
    double lu[MAXD] = {0, 0}, lT;
    if (F->seeded) {
        for (int a = 0; a < D; ++a) lu[a] = F->su[a];
        lT = F->sT;
    } else {
        for (int a = 0; a < D; ++a) lu[a] = mu_[a];
        lT = mT;
    }
    int restarted = !F->seeded;

    double Pf[12][MAXQ], Pg[12][MAXQ], fb[MAXQ], gb[MAXQ], v[MAXQ][MAXD];
    tensors Mfb, Mgb;
    int it, conv = 0, failed = 0, have_pp = 0;
    double pu[MAXD] = {0, 0}, pT = 1.0; /* frame two iterations back */
    double nu[MAXD] = {0, 0}, nT = lT;
    for (it = 1; it <= s->cfg.max_iter; ++it) {
        /* transform every stencil cell into the current frame lambda_k */
        for (int k = 0; k < ns; ++k) {
            project_f(&s->L, s->cfg.reg, &Mf[k], lu, lT, Pf[k]);
            grad_project(&s->L, 2, &Mg[k], lu, lT, Pg[k]);
        }
        velocities(&s->L, lu, lT, v);
        for (int i = 0; i < Q; ++i) {
            /* upwind cell and departure point x' = x_b - v_i dt/2 (MUSCL, Sec. III.B.3) */
            int up = (v[i][axis] >= 0.0);
            int cU = up ? 1 : 2;
            int cB = up ? 0 : 1; /* backward neighbour along the axis */
            int cF = up ? 2 : 3; /* forward neighbour along the axis  */
            double off_a = (up ? 0.5 * s->dx[axis] : -0.5 * s->dx[axis]) - v[i][axis] * h;
            if (fabs(v[i][axis]) * h > 0.5 * s->dx[axis]) ++*depout;
            double sf = orc_limiter(s->cfg.limiter, (Pf[cU][i] - Pf[cB][i]) / s->dx[axis],
                                    (Pf[cF][i] - Pf[cU][i]) / s->dx[axis]);
            double sg = orc_limiter(s->cfg.limiter, (Pg[cU][i] - Pg[cB][i]) / s->dx[axis],
                                    (Pg[cF][i] - Pg[cU][i]) / s->dx[axis]);
            fb[i] = Pf[cU][i] + off_a * sf;
            gb[i] = Pg[cU][i] + off_a * sg;
            for (int q = 0; q < nt; ++q) {
                const int t_axis = t_axes[q], b = 4 + 4 * q;
                int tm = up ? b : b + 2, tp = up ? b + 1 : b + 3;
                double off_t = -v[i][t_axis] * h;
                if (fabs(v[i][t_axis]) * h > 0.5 * s->dx[t_axis]) ++*depout;
                double tf = orc_limiter(s->cfg.limiter, (Pf[cU][i] - Pf[tm][i]) / s->dx[t_axis],
                                        (Pf[tp][i] - Pf[cU][i]) / s->dx[t_axis]);
                double tg = orc_limiter(s->cfg.limiter, (Pg[cU][i] - Pg[tm][i]) / s->dx[t_axis],
                                        (Pg[tp][i] - Pg[cU][i]) / s->dx[t_axis]);
                fb[i] += off_t * tf;
                gb[i] += off_t * tg;
            }
        }
        /* density, momentum and energy at the face -> corrector frame lambda_{k+1} */
        moments(&s->L, fb, lu, lT, &Mfb);
        moments(&s->L, gb, lu, lT, &Mgb);
        double rho = Mfb.t0, ke = 0.0, tr = 0.0;
        for (int a = 0; a < D; ++a) {
            nu[a] = Mfb.t1[a] / rho;
            ke += nu[a] * nu[a];
            tr += Mfb.t2[a][a];
        }
        nT = ((0.5 * tr + Mgb.t0) / rho - 0.5 * ke) / s->Cv;
        if (!(rho > 0.0) || !(nT > 0.0) || !isfinite(nT) || !isfinite(ke)) {
            /* the corrector left the physical states: restart once from the frame of
             * the mean conserved variables of the two neighbours */
            if (!restarted) {
                restarted = 1;
                for (int a = 0; a < D; ++a) lu[a] = mu_[a];
                lT = mT;
                have_pp = 0;
                continue;
            }
            failed = 1;
            break;
        }
        double du = 0.0, du2 = 0.0;
        for (int a = 0; a < D; ++a) {
            du = fmax(du, fabs(nu[a] - lu[a]));
            du2 = fmax(du2, fabs(nu[a] - pu[a]));
        }
        double delta = fmax(du / sqrt(nT), fabs(nT - lT) / nT);
        /* distance to the frame two iterations back: a 2-cycle returns to it */
        double delta2 = fmax(du2 / sqrt(nT), fabs(nT - pT) / nT);
        for (int a = 0; a < D; ++a) {
            pu[a] = lu[a];
            lu[a] = nu[a];
        }
        pT = lT;
        lT = nT;
        if (delta <= s->cfg.tol) {
            conv = 1;
            break;
        }
        if (have_pp && delta2 <= 1e-2 * delta) break; /* oscillation: stop, not converged */
        have_pp = 1;
    }
    if (it > s->cfg.max_iter) it = s->cfg.max_iter;
    F->iters = conv ? it : -it;

    double rho_b = Mfb.t0;
    int has_frame = 1;
    if (failed || !conv) {
        /* Reading (the paper is silent on an iteration that does not converge or leaves
         * the physical states twice): the face takes the first-order upwind state in
         * which every population comes from the neighbour it leaves, in that neighbour's
         * own frame (no common frame, no slope). Its moments give the face frame when
         * they are physical. The last iterate of a non-converged iteration is not used:
         * it depends on the path (a cycle or a wandering sequence), this state does not. */
        ++*nonphys;
        double vL[MAXQ][MAXD], vR[MAXQ][MAXD], hf[MAXQ], hg[MAXQ];
        tensors A, B;
        velocities(&s->L, cL->u, cL->T, vL);
        velocities(&s->L, cR->u, cR->T, vR);
        for (int i = 0; i < Q; ++i) {
            hf[i] = (vL[i][axis] >= 0.0) ? cL->f[i] : 0.0;
            hg[i] = (vL[i][axis] >= 0.0) ? cL->g[i] : 0.0;
        }
        moments(&s->L, hf, cL->u, cL->T, &Mfb);
        moments(&s->L, hg, cL->u, cL->T, &Mgb);
        for (int i = 0; i < Q; ++i) {
            hf[i] = (vR[i][axis] < 0.0) ? cR->f[i] : 0.0;
            hg[i] = (vR[i][axis] < 0.0) ? cR->g[i] : 0.0;
        }
        moments(&s->L, hf, cR->u, cR->T, &A);
        moments(&s->L, hg, cR->u, cR->T, &B);
        Mfb.t0 += A.t0;
        Mgb.t0 += B.t0;
        for (int a = 0; a < D; ++a) {
            Mfb.t1[a] += A.t1[a];
            Mgb.t1[a] += B.t1[a];
            for (int b = 0; b < D; ++b) {
                Mfb.t2[a][b] += A.t2[a][b];
                Mgb.t2[a][b] += B.t2[a][b];
                for (int c = 0; c < D; ++c) Mfb.t3[a][b][c] += A.t3[a][b][c];
            }
        }
        rho_b = Mfb.t0;
        double ke = 0.0, tr = 0.0;
        for (int a = 0; a < D; ++a) {
            nu[a] = Mfb.t1[a] / rho_b;
            ke += nu[a] * nu[a];
            tr += Mfb.t2[a][a];
        }
        nT = ((0.5 * tr + Mgb.t0) / rho_b - 0.5 * ke) / s->Cv;
        if (rho_b > 0.0 && nT > 0.0 && isfinite(nT) && isfinite(ke)) {
            for (int a = 0; a < D; ++a) lu[a] = nu[a];
            lT = nT;
        } else {
            /* no physical face frame: keep the mean frame as the next seed and leave the
             * face populations unrelaxed */
            has_frame = 0;
            for (int a = 0; a < D; ++a) lu[a] = mu_[a];
            lT = mT;
        }
    }

    /* recover phi at the face from phi-bar with the exact co-moving equilibrium of the
     * final face frame (Sec. III.B.3), done on the moments (the map is linear) */
    double eps_b = has_frame ? dt * rho_b * lT / s->cfg.mu : 0.0;
    cellrec eq;
    tensors Mfe, Mge;
    set_equilibrium(s, &eq, rho_b, lu, lT);
    moments(&s->L, eq.f, lu, lT, &Mfe);
    moments(&s->L, eq.g, lu, lT, &Mge);
    tensors Mfo, Mgo;
    memset(&Mfo, 0, sizeof(Mfo));
    memset(&Mgo, 0, sizeof(Mgo));
    Mfo.t0 = orc_face_recover(Mfb.t0, Mfe.t0, eps_b);
    Mgo.t0 = orc_face_recover(Mgb.t0, Mge.t0, eps_b);
    for (int a = 0; a < D; ++a) {
        Mfo.t1[a] = orc_face_recover(Mfb.t1[a], Mfe.t1[a], eps_b);
        Mgo.t1[a] = orc_face_recover(Mgb.t1[a], Mge.t1[a], eps_b);
        for (int b = 0; b < D; ++b) {
            Mfo.t2[a][b] = orc_face_recover(Mfb.t2[a][b], Mfe.t2[a][b], eps_b);
            Mgo.t2[a][b] = orc_face_recover(Mgb.t2[a][b], Mge.t2[a][b], eps_b);
            for (int c = 0; c < D; ++c)
                Mfo.t3[a][b][c] = orc_face_recover(Mfb.t3[a][b][c], Mfe.t3[a][b][c], eps_b);
        }
    }
    pack(D, 3, &Mfo, F->Mf);
    pack(D, 2, &Mgo, F->Mg);
    for (int a = 0; a < D; ++a) F->u[a] = lu[a];
    F->T = lT;
}

/* ------------------------------------------------------------------------- */
/* one time step (Sec. III.B.4)                                              */
/* ------------------------------------------------------------------------- */

/* time step from CFL = max |v_ia| dt / dx_a (Sec. IV) over the cells (in their own frames)
 * and the prescribed boundary states, clipped at t_end */
static double time_step(const orc_sim *s, double t_end)
{
    const int D = s->D, Q = s->Q, nx = s->nx, ny = s->ny, nz = s->nz;
    const double cmax = s->L.c[Q - 1][0]; /* largest node, sqrt(3 + sqrt 6) */
    double rate = 0.0;
#pragma omp parallel for collapse(3) reduction(max : rate) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const cellrec *c = &s->cell[cidx3(s, i, j, k)];
                for (int a = 0; a < D; ++a) {
                    double r = (fabs(c->u[a]) + sqrt(c->T / TL) * cmax) / s->dx[a];
                    rate = fmax(rate, r);
                }
            }
    /* the prescribed boundary states stream into the domain through the boundary faces,
     * so their particle speeds belong to the same maximum (3D has no prescribed states) */
    for (int side = 0; side < 2 * D && side < 4; ++side) {
        int kind = s->cfg.bc[side];
        const double *used[2] = {NULL, NULL};
        if (kind == ORC_BC_FIXED || kind == ORC_BC_SPLIT_FIXED_REFLECT)
            used[0] = s->cfg.bc_state[side];
        if (kind == ORC_BC_FIXED_WINDOW || kind == ORC_BC_MOVING_SHOCK) {
            used[0] = s->cfg.bc_state[side];
            used[1] = s->cfg.bc_alt[side];
        }
        for (int k = 0; k < 2; ++k) {
            if (!used[k]) continue;
            double T = used[k][3] / used[k][0];
            for (int a = 0; a < D; ++a)
                rate = fmax(rate, (fabs(used[k][1 + a]) + sqrt(T / TL) * cmax) / s->dx[a]);
        }
    }
    double dt = s->cfg.cfl / rate;
    if (s->t + dt > t_end) dt = t_end - s->t;
    return dt;
}

/* ------------------------------------------------------------------------- */
/* the semi-Lagrangian realization (Sec. III.A), 1D and 2D                  */
/* ------------------------------------------------------------------------- */

/* Readings (the paper's interpolation recipe is in a cited thesis, not in the paper):
 *  - collocation points are the cell centres; a population is interpolated at its
 *    departure point from the 4 collocation points around it along each axis (2 on each
 *    side: 4 in 1D, the 4 x 4 centres around it in 2D), all of them transformed into the
 *    current frame by the regularized transformation;
 *  - the 4-point kernel is the interpolating cubic (Catmull-Rom) spline, in 2D its tensor
 *    product (the 1D kernel along x, then along y); the limiter clips the value into the
 *    range of the collocation points that enclose the departure point (the two around it
 *    in 1D, the four corners of the square of centres around it in 2D);
 *  - the frame iteration starts from the cell's own frame of the previous step (the
 *    paper's seed) and stops as the face iteration does (tolerance, 2-cycle, max_iter);
 *    a cell whose iteration does not converge keeps its last advected populations;
 *  - the collision is the BGK map of Sec. III.A in the frame of the last advection, with
 *    2 beta = 2 dt / (2 tau + dt), tau = mu / p, i.e. the same relaxation time as the
 *    finite-volume scheme. */
static void catmull_rom(double t, double w[4])
{
    const double t2 = t * t, t3 = t2 * t;
    w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
    w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
    w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
    w[3] = 0.5 * (t3 - t2);
}

/* one cell (ci, cj): frame iteration of the advection, then the collision; writes the new
 * populations (and their frame) into *out. The stencil is the 5 (1D) or 5 x 5 (2D) cells
 * centred on the cell, stencil slot a + 5 b holding cell (ci - 2 + a, cj - 2 + b). */
static void sl_cell(const orc_sim *s, int ci, int cj, double dt, cellrec *out, int *iters, int *conv_out,
                    long long *depout)
{
    const int Q = s->Q, D = s->D;
    const int nst = (D == 1) ? 5 : 25;
    tensors Mf[25], Mg[25];
    for (int b = 0; b < (D == 1 ? 1 : 5); ++b)
        for (int a = 0; a < 5; ++a) {
            const cellrec *c = &s->plus[cidx(s, ci - 2 + a, D == 1 ? 0 : cj - 2 + b)];
            moments(&s->L, c->f, c->u, c->T, &Mf[a + 5 * b]);
            moments(&s->L, c->g, c->u, c->T, &Mg[a + 5 * b]);
        }
    const cellrec *own = &s->plus[cidx(s, ci, D == 1 ? 0 : cj)];
    double lu[MAXD] = {own->u[0], D == 2 ? own->u[1] : 0.0, 0.0}, lT = own->T;
    double pu[MAXD] = {0.0, 0.0, 0.0}, pT = 1.0;
    double fa[MAXQ], ga[MAXQ], fu[MAXD] = {lu[0], lu[1], 0.0}, fT = lT;
    int it, conv = 0, have_pp = 0;
    for (it = 1; it <= s->cfg.max_iter; ++it) {
        double Pf[25][MAXQ], Pg[25][MAXQ], v[MAXQ][MAXD];
        for (int k = 0; k < nst; ++k) {
            project_f(&s->L, s->cfg.reg, &Mf[k], lu, lT, Pf[k]);
            grad_project(&s->L, 2, &Mg[k], lu, lT, Pg[k]);
        }
        velocities(&s->L, lu, lT, v);
        for (int i = 0; i < Q; ++i) {
            /* departure point x_c - v_i dt, in cells along each axis: each component lies in
             * (-1, 1) while the CFL rule holds; base cell c + m, fraction d - m in [0, 1) */
            double w[2][4];
            int m[2] = {0, 0}, out_of_cell = 0;
            for (int ax = 0; ax < D; ++ax) {
                const double d = -v[i][ax] * dt / s->dx[ax];
                if (fabs(d) >= 1.0) out_of_cell = 1;
                m[ax] = (d < 0.0) ? -1 : 0;
                catmull_rom(d - m[ax], w[ax]);
            }
            if (out_of_cell) ++*depout;
            if (D == 1) {
                const int o = m[0];
                double vf = 0.0, vg = 0.0;
                for (int q = 0; q < 4; ++q) {
                    vf += w[0][q] * Pf[o + 1 + q][i];
                    vg += w[0][q] * Pg[o + 1 + q][i];
                }
                const double f1 = Pf[o + 2][i], f2 = Pf[o + 3][i];
                const double g1 = Pg[o + 2][i], g2 = Pg[o + 3][i];
                fa[i] = fmin(fmax(vf, fmin(f1, f2)), fmax(f1, f2));
                ga[i] = fmin(fmax(vg, fmin(g1, g2)), fmax(g1, g2));
            } else {
                /* along x in each of the 4 rows, then along y */
                double vf = 0.0, vg = 0.0;
                for (int qy = 0; qy < 4; ++qy) {
                    double rf = 0.0, rg = 0.0;
                    for (int qx = 0; qx < 4; ++qx) {
                        const int k = (m[0] + 1 + qx) + 5 * (m[1] + 1 + qy);
                        rf += w[0][qx] * Pf[k][i];
                        rg += w[0][qx] * Pg[k][i];
                    }
                    vf += w[1][qy] * rf;
                    vg += w[1][qy] * rg;
                }
                double flo = INFINITY, fhi = -INFINITY, glo = INFINITY, ghi = -INFINITY;
                for (int cy = 0; cy < 2; ++cy)
                    for (int cx = 0; cx < 2; ++cx) {
                        const int k = (m[0] + 2 + cx) + 5 * (m[1] + 2 + cy);
                        flo = fmin(flo, Pf[k][i]);
                        fhi = fmax(fhi, Pf[k][i]);
                        glo = fmin(glo, Pg[k][i]);
                        ghi = fmax(ghi, Pg[k][i]);
                    }
                fa[i] = fmin(fmax(vf, flo), fhi);
                ga[i] = fmin(fmax(vg, glo), ghi);
            }
        }
        for (int a = 0; a < D; ++a) fu[a] = lu[a];
        fT = lT;
        double rho, nu[MAXD] = {0, 0, 0}, nT;
        macro(s, fa, ga, lu, lT, &rho, nu, &nT);
        if (!(rho > 0.0) || !(nT > 0.0) || !isfinite(nT)) break; /* the cell fails */
        double du = 0.0, du2 = 0.0;
        for (int a = 0; a < D; ++a) {
            du = fmax(du, fabs(nu[a] - lu[a]));
            du2 = fmax(du2, fabs(nu[a] - pu[a]));
        }
        double delta = fmax(du / sqrt(nT), fabs(nT - lT) / nT);
        double delta2 = fmax(du2 / sqrt(nT), fabs(nT - pT) / nT);
        for (int a = 0; a < D; ++a) {
            pu[a] = lu[a];
            lu[a] = nu[a];
        }
        pT = lT;
        lT = nT;
        if (delta <= s->cfg.tol) {
            conv = 1;
            break;
        }
        if (have_pp && delta2 <= 1e-2 * delta) break; /* 2-cycle */
        have_pp = 1;
    }
    if (it > s->cfg.max_iter) it = s->cfg.max_iter;
    *iters = it;
    *conv_out = conv;
    /* collision in the frame of the last advection (Sec. III.A) */
    double rho = 0.0;
    for (int i = 0; i < Q; ++i) rho += fa[i];
    const double eps = dt * rho * fT / s->cfg.mu;
    const double b2 = 2.0 * eps / (2.0 + eps); /* 2 beta */
    const double geq = (s->Cv - 0.5 * D) * rho * fT;
    for (int i = 0; i < Q; ++i) {
        out->f[i] = fa[i] + b2 * (rho * s->L.W[i] - fa[i]);
        out->g[i] = ga[i] + b2 * (geq * s->L.W[i] - ga[i]);
    }
    out->u[0] = fu[0];
    out->u[1] = fu[1];
    out->T = fT;
    out->rho = rho;
}

static int sl_step(orc_sim *s, double t_end, orc_stats *st)
{
    const int nx = s->nx, ny = (s->D == 1) ? 1 : s->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            cellrec tmp;
            reframe_cell(s, &s->cell[cidx(s, i, j)], &tmp);
            s->cell[cidx(s, i, j)] = tmp;
        }
    const double dt = time_step(s, t_end);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) s->plus[cidx(s, i, j)] = s->cell[cidx(s, i, j)];
    fill_ghosts(s);
    long long itot = 0, nonc = 0, depout = 0;
    int imax = 0;
#pragma omp parallel for collapse(2) reduction(+ : itot, nonc, depout) reduction(max : imax) schedule(dynamic, 16)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int it, conv;
            sl_cell(s, i, j, dt, &s->cell[cidx(s, i, j)], &it, &conv, &depout);
            itot += it;
            if (it > imax) imax = it;
            if (!conv) ++nonc;
        }
    s->t += dt;
    s->nstep += 1;
    if (st) {
        st->faces = (long long)nx * ny;
        st->iters_total = itot;
        st->iters_max = imax;
        st->nonconverged = nonc;
        st->departure_out = depout;
        st->nonphysical = 0;
        st->dt = dt;
    }
    return nonc ? 2 : 0;
}

/* face index of the face on the `hi` side of cell (i, j, k) along `axis` */
static long long face_of(const orc_sim *s, int axis, int i, int j, int k, int hi)
{
    if (axis == 0) return (long long)(i + hi) + (long long)(s->nx + 1) * (j + (long long)s->ny * k);
    if (axis == 1) return s->nfx + (long long)i + (long long)s->nx * ((j + hi) + (long long)(s->ny + 1) * k);
    return s->nfx + s->nfy + (long long)i + (long long)s->nx * (j + (long long)s->ny * (k + hi));
}

int orc_step(orc_sim *s, double t_end, orc_stats *st)
{
    const int D = s->D, Q = s->Q, nx = s->nx, ny = s->ny, nz = s->nz;
    if (s->t >= t_end) return 1;
    if (s->cfg.scheme == ORC_SCHEME_SL) return sl_step(s, t_end, st);

    /* 1. every cell's populations in its own co-moving frame */
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                cellrec tmp;
                reframe_cell(s, &s->cell[cidx3(s, i, j, k)], &tmp);
                s->cell[cidx3(s, i, j, k)] = tmp;
            }

    double dt = time_step(s, t_end);

    /* 2. phi-bar-plus of every cell (Sec. III.B.3), eps = dt/tau = dt p / mu */
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const cellrec *c = &s->cell[cidx3(s, i, j, k)];
                cellrec *o = &s->plus[cidx3(s, i, j, k)];
                double eps = dt * c->rho * c->T / s->cfg.mu;
                double geq_coef = (s->Cv - 0.5 * D) * c->T * c->rho;
                for (int q = 0; q < Q; ++q) {
                    o->f[q] = orc_phibar_plus(c->f[q], c->rho * s->L.W[q], eps);
                    o->g[q] = orc_phibar_plus(c->g[q], geq_coef * s->L.W[q], eps);
                }
                for (int a = 0; a < D; ++a) o->u[a] = c->u[a];
                o->T = c->T;
                o->rho = c->rho;
            }
    fill_ghosts(s);

    /* 3. faces: predictor-corrector frame iteration and face moments */
    long long depout = 0, nonphys = 0;
#pragma omp parallel for collapse(3) reduction(+ : depout, nonphys) schedule(dynamic, 16)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i)
                face_iteration(s, &s->face[face_of(s, 0, i - 1, j, k, 1)], 0, i - 1, j, k, dt, &depout, &nonphys);
    if (D >= 2) {
#pragma omp parallel for collapse(3) reduction(+ : depout, nonphys) schedule(dynamic, 16)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i < nx; ++i)
                    face_iteration(s, &s->face[face_of(s, 1, i, j - 1, k, 1)], 1, i, j - 1, k, dt, &depout, &nonphys);
    }
    if (D == 3) {
#pragma omp parallel for collapse(3) reduction(+ : depout, nonphys) schedule(dynamic, 16)
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i)
                    face_iteration(s, &s->face[face_of(s, 2, i, j, k - 1, 1)], 2, i, j, k - 1, dt, &depout, &nonphys);
    }

    /* 4. flux into each cell's frame and the co-moving update (Sec. III.B.2) */
#pragma omp parallel for collapse(3) schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                cellrec *c = &s->cell[cidx3(s, i, j, k)];
                double v[MAXQ][MAXD];
                velocities(&s->L, c->u, c->T, v);
                double Ff[MAXQ], Fg[MAXQ];
                for (int q = 0; q < Q; ++q) Ff[q] = Fg[q] = 0.0;
                for (int a = 0; a < D; ++a)
                    for (int side = 0; side < 2; ++side) {
                        /* side 0: face at x_j - dx/2 with outward normal -e_a; side 1: +e_a */
                        const facerec *F = &s->face[face_of(s, a, i, j, k, side)];
                        tensors Mf, Mg;
                        unpack(D, 3, F->Mf, &Mf);
                        unpack(D, 2, F->Mg, &Mg);
                        double pf[MAXQ], pg[MAXQ];
                        project_f(&s->L, s->cfg.reg, &Mf, c->u, c->T, pf);
                        grad_project(&s->L, 2, &Mg, c->u, c->T, pg);
                        double nsign = side ? 1.0 : -1.0;
                        for (int q = 0; q < Q; ++q) {
                            /* (dt/V_j) A_c (v_i . n_c) phi_i = (dt/dx_a) (+-v_ia) phi_i */
                            Ff[q] += dt / s->dx[a] * nsign * v[q][a] * pf[q];
                            Fg[q] += dt / s->dx[a] * nsign * v[q][a] * pg[q];
                        }
                    }
                double eps = dt * c->rho * c->T / s->cfg.mu;
                double geq_coef = (s->Cv - 0.5 * D) * c->T * c->rho;
                for (int q = 0; q < Q; ++q) {
                    c->f[q] = orc_update_relax(c->f[q], c->rho * s->L.W[q], eps) - Ff[q];
                    c->g[q] = orc_update_relax(c->g[q], geq_coef * s->L.W[q], eps) - Fg[q];
                }
                /* the updated populations stay in the frame lambda_j(t_n) */
            }

    /* face frames seed the next step's predictor */
    long long nf = s->nfx + s->nfy + s->nfz, itot = 0, nonc = 0;
    int imax = 0;
    for (long long q = 0; q < nf; ++q) {
        facerec *F = &s->face[q];
        for (int a = 0; a < D; ++a) F->su[a] = F->u[a];
        F->sT = F->T;
        F->seeded = 1;
        int it = F->iters < 0 ? -F->iters : F->iters;
        itot += it;
        if (it > imax) imax = it;
        if (F->iters < 0) ++nonc;
    }
    s->t += dt;
    s->nstep += 1;
    if (st) {
        st->faces = nf;
        st->iters_total = itot;
        st->iters_max = imax;
        st->nonconverged = nonc;
        st->departure_out = depout;
        st->nonphysical = nonphys;
        st->dt = dt;
    }
    return nonc ? 2 : 0;
}

/* ------------------------------------------------------------------------- */
/* read-out                                                                  */
/* ------------------------------------------------------------------------- */

/* cell (i, j, k) of the interior, x fastest: its storage record and its output index */
#define FOR_CELLS(s)                                                                               \
    for (int kz_ = 0; kz_ < (s)->nz; ++kz_)                                                        \
        for (int j_ = 0; j_ < (s)->ny; ++j_)                                                       \
            for (int i_ = 0; i_ < (s)->nx; ++i_)
#define CELL_OUT(s) ((long long)i_ + (long long)(s)->nx * (j_ + (long long)(s)->ny * kz_))
#define CELL_REC(s) (&(s)->cell[cidx3((s), i_, j_, kz_)])

void orc_fields(const orc_sim *s, double *rho, double *ux, double *uy, double *T)
{
    FOR_CELLS(s) {
        const cellrec *c = CELL_REC(s);
        long long k = CELL_OUT(s);
        double r, u[MAXD] = {0, 0, 0}, t;
        macro(s, c->f, c->g, c->u, c->T, &r, u, &t);
        rho[k] = r;
        ux[k] = u[0];
        if (uy && s->D >= 2) uy[k] = u[1];
        T[k] = t;
    }
}

void orc_conserved(const orc_sim *s, double *U)
{
    long long n = (long long)s->nx * s->ny * s->nz;
    FOR_CELLS(s) {
        const cellrec *c = CELL_REC(s);
        long long k = CELL_OUT(s);
        tensors Mf, Mg;
        moments(&s->L, c->f, c->u, c->T, &Mf);
        moments(&s->L, c->g, c->u, c->T, &Mg);
        double tr = 0.0;
        U[k] = Mf.t0;
        for (int a = 0; a < s->D; ++a) {
            U[(1 + a) * n + k] = Mf.t1[a];
            tr += Mf.t2[a][a];
        }
        U[(1 + s->D) * n + k] = 0.5 * tr + Mg.t0;
    }
}

static void copy_out(const orc_sim *s, const cellrec *c, long long k, long long n, double *f,
                     double *g, double *frame)
{
    for (int q = 0; q < s->Q; ++q) {
        if (f) f[q * n + k] = c->f[q];
        if (g) g[q * n + k] = c->g[q];
    }
    if (frame) {
        for (int a = 0; a < s->D; ++a) frame[a * n + k] = c->u[a];
        frame[s->D * n + k] = c->T;
    }
}

void orc_populations(const orc_sim *s, double *f, double *g, double *frame)
{
    long long n = (long long)s->nx * s->ny * s->nz;
    FOR_CELLS(s) copy_out(s, CELL_REC(s), CELL_OUT(s), n, f, g, frame);
}

void orc_reframed(const orc_sim *s, double *f, double *g, double *frame)
{
    long long n = (long long)s->nx * s->ny * s->nz;
    FOR_CELLS(s) {
        cellrec tmp;
        reframe_cell(s, CELL_REC(s), &tmp);
        copy_out(s, &tmp, CELL_OUT(s), n, f, g, frame);
    }
}

void orc_face_frames(const orc_sim *s, double *out)
{
    long long nf = s->nfx + s->nfy + s->nfz;
    for (long long k = 0; k < nf; ++k) {
        for (int a = 0; a < s->D; ++a) out[k * (s->D + 1) + a] = s->face[k].su[a];
        out[k * (s->D + 1) + s->D] = s->face[k].sT;
    }
}

void orc_set_face_frames(orc_sim *s, const double *in)
{
    long long nf = s->nfx + s->nfy + s->nfz;
    for (long long k = 0; k < nf; ++k) {
        for (int a = 0; a < s->D; ++a) s->face[k].su[a] = in[k * (s->D + 1) + a];
        s->face[k].sT = in[k * (s->D + 1) + s->D];
        s->face[k].seeded = 1;
    }
}

void orc_face_moments(const orc_sim *s, double *Mf, double *Mg)
{
    const int D = s->D;
    const int nf3 = 1 + D + D * D + D * D * D, ng2 = 1 + D + D * D;
    long long nf = s->nfx + s->nfy + s->nfz;
    for (long long k = 0; k < nf; ++k) {
        for (int q = 0; q < nf3; ++q) Mf[k * nf3 + q] = s->face[k].Mf[q];
        for (int q = 0; q < ng2; ++q) Mg[k * ng2 + q] = s->face[k].Mg[q];
    }
}

void orc_face_iters(const orc_sim *s, int *out)
{
    long long nf = s->nfx + s->nfy + s->nfz;
    for (long long k = 0; k < nf; ++k) out[k] = s->face[k].iters;
}
