/*
 * pond_oracle.h -- C interface of the plain FP64 CPU oracle of the finite-volume
 * Particles-on-Demand (PonD) time step (Kallikounis, Dorschner & Karlin,
 * "Particles on Demand for flows with strong discontinuities").
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library. It shares no code, header, table or constant
 * with the GPU library (include/pond.h and the HIP sources).
 *
 * Units: gas constant R = 1 (p = rho T), lattice temperature T_L = 1.
 */
#ifndef POND_ORACLE_H
#define POND_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds, per side (west, east, south, north) */
enum {
    ORC_BC_PERIODIC = 0,
    ORC_BC_OUTFLOW = 1,      /* zero gradient: ghost = nearest interior cell            */
    ORC_BC_REFLECT = 2,      /* mirror cell, normal velocity reversed                   */
    ORC_BC_FIXED = 3,        /* equilibrium at bc_state                                 */
    ORC_BC_FIXED_WINDOW = 4, /* bc_alt where lo <= tangential centre <= hi, else bc_state */
    ORC_BC_SPLIT_FIXED_REFLECT = 5, /* fixed bc_state for tangential centre < param[0], reflect beyond */
    ORC_BC_MOVING_SHOCK = 6  /* bc_state if x_c < p0 + p1*(y_c + p2*t), else bc_alt       */
};

enum { ORC_LIM_VANLEER = 0, ORC_LIM_MINMOD = 1 };

/* regularization of the f-populations in a change of frame (Sec. II.C): third-order Grad
 * projection (the paper's choice), or the alternative that keeps the moments of order
 * 0..3 and sets the other Q - q moments to equilibrium by moment inversion (D2Q16 only;
 * in 1D, D1Q4 has no other moments and both are the same). */
enum { ORC_REG_GRAD = 0, ORC_REG_EQ = 1 };

/* discretization: the finite-volume scheme (Sec. III.B, the paper's main one) or the
 * semi-Lagrangian realization (Sec. III.A; 1D and 2D here) */
enum { ORC_SCHEME_FV = 0, ORC_SCHEME_SL = 1 };

typedef struct {
    int dim;              /* 1 or 2                                   */
    int nx, ny;           /* interior cells (ny = 1 in 1D)            */
    double x0, x1, y0, y1;
    double gamma;         /* adiabatic exponent, C_v = 1/(gamma-1)    */
    double cfl;           /* max |v_ia| dt/dx                         */
    double mu;            /* dynamic viscosity, tau = mu/p            */
    int limiter;          /* ORC_LIM_*                                */
    double tol;           /* frame convergence tolerance              */
    int max_iter;         /* iteration cap per face                   */
    int bc[4];            /* west, east, south, north                 */
    double bc_state[4][4];/* rho, ux, uy, p                           */
    double bc_alt[4][4];  /* second state (window / pre-shock)        */
    double bc_param[4][4];/* geometry parameters                      */
    int reg;              /* ORC_REG_*                                */
    int scheme;           /* ORC_SCHEME_*                             */
    /* 3D (dim 3, D3Q64): cells along z, the z extent, and the kinds of the two z sides
     * (bottom, top); 3D takes the periodic, outflow and reflecting kinds only, and the
     * Grad projection of the finite-volume scheme */
    int nz;
    double z0, z1;
    int bc_z[2];
} orc_config;

typedef struct {
    long long faces;          /* faces processed                        */
    long long iters_total;    /* sum of iterations over faces           */
    int iters_max;
    long long nonconverged;   /* faces that hit max_iter                */
    long long departure_out;  /* populations whose departure point left the upwind cell */
    long long nonphysical;    /* faces that fell back to the upwind state in own frames */
    double dt;                /* last time step                         */
} orc_stats;

typedef struct orc_sim orc_sim;

/* the ORC_REG_EQ transformation of populations with lab moments M (packed as for
 * orc_grad_project, order 3) into frame {u, T}: f has Q entries */
void orc_eq_project(int dim, const double *M, const double *u, double T, double *f);

/* lattice of Table I: D1Q4 (dim 1) or D2Q16 (dim 2), and its tensor product D3Q64 (dim 3).
 * c: Q*dim, W: Q. returns Q */
int orc_lattice(int dim, double *c, double *W);

/* lab-frame moment tensors M_0..M_order of populations f expressed in frame (u, T);
 * packed as [M0, M1(dim), M2(dim*dim), M3(dim^3)] (only up to `order`). */
void orc_moments(int dim, int order, const double *f, const double *u, double T, double *M);

/* Grad projection of order 2 or 3 with moments M (packed as above) into frame (u, T) */
void orc_grad_project(int dim, int order, const double *M, const double *u, double T, double *f);

/* Grad coefficients a_0..a_order (packed like the moments) */
void orc_grad_coefficients(int dim, int order, const double *M, const double *u, double T, double *a);

double orc_limiter(int kind, double backward, double forward);

/* phi-bar-plus, face recovery and cell update maps applied to one population */
double orc_phibar_plus(double ftilde, double feq, double eps);
double orc_face_recover(double phibar, double feq, double eps_face);
double orc_update_relax(double ftilde, double feq, double eps);

orc_sim *orc_create(const orc_config *cfg, const double *rho, const double *ux,
                    const double *uy, const double *p);
/* the same with the z velocity (3D; uz may be NULL in 1D and 2D) */
orc_sim *orc_create3(const orc_config *cfg, const double *rho, const double *ux,
                     const double *uy, const double *uz, const double *p);
void orc_destroy(orc_sim *s);

/* advance one step (dt clipped so that t does not pass t_end); returns 0 on success,
 * 1 if t >= t_end already (nothing done), 2 if some face did not converge */
int orc_step(orc_sim *s, double t_end, orc_stats *st);
double orc_time(const orc_sim *s);
long long orc_steps(const orc_sim *s);

/* interior fields rho, ux, uy, T from the conserved moments (uy may be NULL in 1D) */
void orc_fields(const orc_sim *s, double *rho, double *ux, double *uy, double *T);
/* conserved variables (rho, rho u..., rho E), plane by plane: (dim+2) x ncells */
void orc_conserved(const orc_sim *s, double *U);
/* stored populations (Q x ncells each) and their frames ((dim+1) x ncells) */
void orc_populations(const orc_sim *s, double *f, double *g, double *frame);
/* the populations after the reframe that opens the next step, and the new frames */
void orc_reframed(const orc_sim *s, double *f, double *g, double *frame);
/* face frames from the last step: x-faces then y-faces, (dim+1) values per face */
void orc_face_frames(const orc_sim *s, double *out);
/* face moments (f: 1+d+d^2+d^3, g: 1+d+d^2 values per face) of the last step */
void orc_face_moments(const orc_sim *s, double *Mf, double *Mg);
/* replace the face seeds (layout of orc_face_frames) */
void orc_set_face_frames(orc_sim *s, const double *in);
/* iteration count per face of the last step */
void orc_face_iters(const orc_sim *s, int *out);
long long orc_nfaces(const orc_sim *s);

int orc_num_threads(void);
/* threads of the OpenMP loops of later calls (n >= 1) */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
