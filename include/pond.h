/*
 * pond.h -- C ABI of libpond, an MI355X (gfx950) implementation of the
 * finite-volume Particles-on-Demand (PonD) time step of Kallikounis, Dorschner &
 * Karlin, "Particles on Demand for flows with strong discontinuities".
 *
 * One step (paper Sec. III.B.4) is:
 *   - every cell's populations expressed in its co-moving frame by the regularized
 *     (Grad) transformation of Sec. II.C: third order for f, second order for g;
 *   - phi-bar-plus of every cell (Sec. III.B.3);
 *   - per face, the predictor-corrector iteration of the face frame with limited
 *     MUSCL reconstruction at the half-step departure points (Sec. III.B.3);
 *   - the face populations converted into each cell's frame, the flux and the
 *     co-moving BGK update (Sec. III.B.2, the update of f~ and g~).
 *
 * Conventions for every entry point:
 *   - units with gas constant 1 (p = rho T) and lattice temperature T_L = 1;
 *     C_v = 1/(gamma - 1); tau = mu / p (Prandtl number 1);
 *   - cell fields are plain arrays in x-fastest order (index i + nx*j, in 3D
 *     i + nx*(j + ny*k));
 *   - host pointers are caller-owned and only read or written during the call;
 *   - device memory is owned by the context; no entry point retains a caller pointer;
 *   - on an error the context keeps the state of the last completed step;
 *   - all calls on one context go to its stream in order; a context is not
 *     thread-safe, distinct contexts are independent.
 */
#ifndef POND_H
#define POND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POND_ABI_VERSION 5

typedef enum {
    POND_OK = 0,
    POND_EINVAL = 1,   /* invalid argument, configuration or initial state      */
    POND_ENOMEM = 2,   /* device allocation failed                              */
    POND_EDEVICE = 3,  /* HIP runtime error or no usable gfx950 device          */
    POND_ENOCONV = 4,  /* some face did not converge within max_iter (reported   */
                       /* by pond_step only when POND_FLAG_STRICT is set)       */
    POND_ECFL = 5,     /* a departure point left its upwind cell                 */
    POND_ENONPHYS = 6, /* rho <= 0, T <= 0 or a non-finite value in a cell       */
    POND_ESTATE = 7    /* call not valid in the context's state                  */
} pond_status;

/* boundary kinds, one per side: west, east, south, north (Sec. IV); in 3D also bottom and
 * top (bc_z), where only the periodic, outflow and reflecting kinds are taken */
enum {
    POND_BC_PERIODIC = 0,
    POND_BC_OUTFLOW = 1,             /* zero gradient: ghost = nearest interior cell      */
    POND_BC_REFLECT = 2,             /* mirrored cell, normal velocity reversed           */
    POND_BC_FIXED = 3,               /* equilibrium at bc_state                           */
    POND_BC_FIXED_WINDOW = 4,        /* bc_alt where param[0] <= tangential centre <=     */
                                     /* param[1], bc_state elsewhere                      */
    POND_BC_SPLIT_FIXED_REFLECT = 5, /* fixed bc_state where the tangential centre is    */
                                     /* below param[0], reflecting beyond                 */
    POND_BC_MOVING_SHOCK = 6         /* bc_state where x_c < p0 + p1 (y_c + p2 t), bc_alt */
                                     /* beyond (a plane shock crossing the boundary)      */
};

enum { POND_LIM_VANLEER = 0, POND_LIM_MINMOD = 1 };
enum { POND_FP64 = 0, POND_MIXED = 1 };    /* MIXED: FP32 populations, FP64 conserved */
enum { POND_SEED_PREV = 0, POND_SEED_MLP = 1 };
enum {
    POND_FLAG_STRICT = 1, /* non-converged faces are an error                              */
    /* the alternative regularization of Sec. II.C for the f populations (2D; in 1D the
     * D1Q4 moments are all kept and it changes nothing): in every change of frame the
     * moments of degree <= 3 are kept and the six other moments of the D2Q16 moment
     * vector (frame-relative monomials c_x^a c_y^b, a, b <= 3, a + b >= 4) take the values
     * of the product-form equilibrium with the state's density and velocity and the new
     * frame's temperature; the populations follow by moment inversion. Default: the
     * third-order Grad projection, the paper's choice. */
    POND_FLAG_REG_EQ = 2,
    /* 1D and 2D: the semi-Lagrangian realization of Sec. III.A instead of the
     * finite-volume scheme: every cell iterates its frame with its populations advected
     * from the departure points x - v_i dt (4-point interpolating cubic kernel over the
     * cell centres, in 2D its tensor product over the 4 x 4 centres, clipped into the
     * range of the centres that enclose the departure point), then relaxes with the BGK
     * collision of that section. Not conservative (the paper's point in favour of the
     * finite-volume scheme). Not with the learned seed or the resident launch, not in 3D
     * (EINVAL). */
    POND_FLAG_SEMI_LAGRANGIAN = 4
};

/* How a 2D context holds each cell's populations between steps (pond_set_state_layout). */
enum {
    /* the non-equilibrium Hermite coefficients of f (7) and g (5) in the cell's own
     * co-moving frame: the projections of Sec. II.C keep exactly these (f to degree 3, g
     * to degree 2), so they determine the 2Q populations (default) */
    POND_LAYOUT_HERMITE = 0,
    /* the 2Q = 32 populations f_i, g_i themselves (Sec. III.B.4: each cell's populations
     * in its own frame), one plane per population */
    POND_LAYOUT_POPULATIONS = 1
};

/* Problem statement (paper Sec. IV: initial fields on a uniform grid, gamma, CFL,
 * viscosity, boundary conditions). Caller-owned, copied by pond_init. */
typedef struct {
    int32_t dim;            /* 1 (D1Q4 lattice) or 2 (D2Q16 lattice), Table I; 3: the   */
                            /* D3Q64 tensor product of D1Q4 (Sec. II.A), 20 moments of  */
                            /* f in the Grad projection (Sec. II.C); pond_init3 only    */
    int32_t nx, ny;         /* cells; in 1D nx is the total over all instances, ny = 1 */
    int32_t n_inst;         /* 1D only: number of independent tubes (>= 1)              */
    const int32_t *len;     /* 1D only: cells per tube (n_inst values, each >= 4), or  */
                            /* NULL for a single tube of nx cells. Read by pond_init.   */
    double x0, x1, y0, y1;  /* domain; every tube spans [x0, x1]                        */
    double gamma;           /* adiabatic exponent (> 1)                                 */
    double cfl;             /* max |v_ia| dt / dx_a, in (0, 1)                          */
    double mu;              /* dynamic viscosity (> 0)                                  */
    int32_t limiter;        /* POND_LIM_*                                               */
    double tol;             /* face-frame convergence tolerance (> 0)                   */
    int32_t max_iter;       /* iteration cap per face (>= 1)                            */
    int32_t precision;      /* POND_FP64 or POND_MIXED                                  */
    int32_t seed_mode;      /* POND_SEED_PREV or POND_SEED_MLP (needs pond_load_mlp)    */
    int32_t flags;          /* POND_FLAG_*                                              */
    int32_t bc[4];          /* west, east, south, north: POND_BC_*                      */
    double bc_state[4][4];  /* per side: rho, ux, uy, p                                 */
    double bc_alt[4][4];    /* second state of the window and moving-shock kinds       */
    double bc_param[4][4];  /* geometry of the window, split and moving-shock kinds     */
    /* 3D only (read when dim == 3): cells along z, the z extent, and the kinds of the
     * bottom and top sides. A 3D context takes the periodic, outflow and reflecting kinds
     * on all six sides, the Grad projection and the finite-volume scheme, the previous
     * face frame as seed (flags 0 or POND_FLAG_STRICT, seed_mode POND_SEED_PREV), and
     * gamma <= 5/3 (C_v >= 3/2); the launch-control calls of the 2D face tiles, the tail
     * hand-over and the resident launch do not apply (POND_EINVAL), pond_autotune leaves a
     * 3D context unchanged. */
    int32_t nz;
    double z0, z1;
    int32_t bc_z[2];
} pond_config;

/* Counters of the steps taken by one pond_step call (all instances together). */
typedef struct {
    int64_t steps;                  /* steps taken (the maximum over instances)        */
    int64_t cell_updates;           /* cells advanced, summed over steps               */
    int64_t converged_cell_updates; /* of which every face met tol within max_iter     */
    int64_t faces;                  /* face iterations started, summed over steps      */
                                    /* (semi-Lagrangian scheme: cell iterations)        */
    int64_t iters_total;            /* frame iterations, summed over faces and steps   */
    int32_t iters_max;              /* largest iteration count of one face             */
    int64_t nonconverged;           /* faces that hit max_iter                         */
    int64_t fallback;               /* faces that used the first-order fallback state  */
    int64_t departure_out;          /* populations whose departure point left the cell */
    double t_min, t_max;            /* time of the instances after the call            */
    double dt_min, dt_max;          /* time steps of the last step over instances      */
    int32_t failed_instances;       /* instances frozen after producing an invalid cell */
    int64_t tail_faces;             /* 2D: faces finished by the tail kernel           */
    int64_t tail_iters;             /* 2D: iterations run by the tail kernel           */
    /* the state after the call (Sec. II.B definitions: rho, T = (E - u^2/2)/C_v from the
     * conserved variables), from one extra pass over cells and faces: */
    double rho_min;                 /* smallest cell density                           */
    double T_min;                   /* smallest cell temperature                       */
    double totals[5];               /* sum over all cells of the conserved variables   */
                                    /* times the cell volume: mass, momentum (dim       */
                                    /* values), energy; unused entries 0                */
    int32_t first_failed_instance;  /* lowest instance that failed in this call, or -1 */
    int64_t first_failed_cell;      /* lowest cell index (x fastest, tubes concatenated) */
                                    /* holding rho <= 0, T <= 0 or a non-finite value,  */
                                    /* or -1                                            */
    int64_t first_nonconv_face;     /* lowest face index whose iteration in the last   */
                                    /* step did not converge (see pond_face_iters), -1 */
} pond_stats;

typedef struct pond_ctx pond_ctx;

/* Create a context: validate cfg, allocate device state and set every cell to the
 * local equilibrium f = rho W_i, g = (C_v - D/2) rho T W_i of its initial state in its
 * co-moving frame {u, T = p/rho} (Sec. II.B). rho, ux, p: host arrays of nx*ny values;
 * uy may be NULL in 1D. rho and p must be positive and finite. On error *out = NULL. */
pond_status pond_init(const pond_config *cfg, const double *rho, const double *ux,
                      const double *uy, const double *p, pond_ctx **out);
/* The same with the z velocity, for every dimension (uz is read in 3D only and may be
 * NULL in 1D and 2D); host arrays of nx*ny*nz values in 3D. pond_init refuses dim 3. */
pond_status pond_init3(const pond_config *cfg, const double *rho, const double *ux,
                       const double *uy, const double *uz, const double *p, pond_ctx **out);

/* Advance every instance by up to nsteps steps of Sec. III.B.4, each with dt = cfl / max
 * rate of its cells (Sec. IV), the last one clipped so that no instance passes t_end (pass
 * INFINITY for a fixed step count). st (may be NULL) receives the counters of this call and
 * the summary of the state after it (one extra pass over cells and faces, skipped when st
 * is NULL). Returns POND_OK, or the first error found in this call (POND_ENONPHYS if one of
 * its steps produced an invalid cell; POND_ECFL and POND_ENOCONV only with
 * POND_FLAG_STRICT); an instance that failed in an earlier call stays frozen and is
 * counted in st->failed_instances, but does not make later calls fail.
 * The call is asynchronous on the context's stream except for the counter read-back. */
pond_status pond_step(pond_ctx *ctx, int32_t nsteps, double t_end, pond_stats *st);

/* Cell fields rho, ux, uy, T computed from the conserved variables (Sec. II.B: u = rho u /
 * rho, T = (E - u^2/2) / C_v); host arrays of nx*ny (nx*ny*nz in 3D, whose z velocity is
 * in pond_conserved); uy may be NULL. Synchronizes the stream. */
pond_status pond_moments(const pond_ctx *ctx, double *rho, double *ux, double *uy, double *T);

/* Same fields (Sec. II.B) written to a caller-owned device buffer of 4*nx*ny doubles
 * (planes rho, ux, uy, T) on the context's stream; does not synchronize. */
pond_status pond_moments_device(const pond_ctx *ctx, double *dev_out);

/* Conserved variables (rho, rho u_x[, rho u_y[, rho u_z]], rho E) of Sec. II.B, the moments
 * the finite-volume update of Sec. III.B.2 conserves: (dim+2) planes of the cell count. */
pond_status pond_conserved(const pond_ctx *ctx, double *U);

/* Populations f~, g~ (the carried variables of Sec. III.B.1, in the Grad form of
 * Sec. II.C; Q planes of nx*ny each, Q = 4^dim) and their frames ((dim+1)
 * planes: u..., T) as the next step starts from them: in each cell's co-moving frame. */
pond_status pond_populations(const pond_ctx *ctx, double *f, double *g, double *frame);

/* Number of faces x_b (the cell interfaces of Sec. III.B.3): 1D: nx + n_inst; 2D: (nx+1)*ny
 * x-faces followed by nx*(ny+1) y-faces (x-face (i,j) lies between cells (i-1,j) and (i,j);
 * y-face (i,j) between (i,j-1), (i,j)); 3D: (nx+1)*ny*nz x-faces (index i + (nx+1)(j +
 * ny k)), nx*(ny+1)*nz y-faces (i + nx (j + (ny+1) k)), nx*ny*(nz+1) z-faces
 * (i + nx (j + ny k)), the face with index i (j, k) along its axis lying between cells
 * i - 1 and i of that axis. */
int64_t pond_nfaces(const pond_ctx *ctx);

/* Face frames lambda_b of the last step (Sec. III.B.3; (dim+1) values per face: u..., T)
 * = the seeds of the next step's predictor. Host array of pond_nfaces*(dim+1). Before the
 * first step every T is -1 (no seed yet). */
pond_status pond_face_frames(const pond_ctx *ctx, double *out);
/* Replace the seeds, the predictor frames lambda_0 of Sec. III.B.3 (same layout). T <= 0
 * marks a face as unseeded. */
pond_status pond_set_face_frames(pond_ctx *ctx, const double *in);
/* Lab-frame moments of the face populations phi(x_b, t+dt/2) of the last step (Sec.
 * III.B.3, after the recovery from phi-bar with the face equilibrium):
 * f: 1+d+d^2+d^3 values (M0, M1, M2, M3 row-major), g: 1+d+d^2 values, per face. */
pond_status pond_face_moments(const pond_ctx *ctx, double *Mf, double *Mg);
/* Iteration count of the predictor-corrector loop of Sec. III.B.3 per face of the last
 * step (negative: not converged; the face then took the first-order fallback state). */
pond_status pond_face_iters(const pond_ctx *ctx, int32_t *out);

/* Per instance (the step of Sec. III.B.4 has no failure handling; this is the library's):
 * nonzero once one of its steps produced a cell with rho <= 0, T <= 0 or a
 * non-finite value. Such an instance is frozen (its later steps have dt = 0) while the
 * other instances go on; pond_step reports POND_ENONPHYS for the call in which it failed. */
pond_status pond_failed_instances(const pond_ctx *ctx, int32_t *flags);

/* Time of each instance, the sum of its time steps (Sec. IV; host array of n_inst). */
pond_status pond_time(const pond_ctx *ctx, double *t);

/* Launch control (changes where the work of Sec. III.B.4 runs, not what it computes).
 * Make the context issue its work on a caller's HIP stream (hipStream_t passed as
 * void*; NULL = the context's own stream). The stream must outlive the context or
 * be replaced before it is destroyed. */
pond_status pond_set_stream(pond_ctx *ctx, void *hip_stream);

/* Launch control (results of Sec. III.B.4 unchanged). Launch shapes. 1D: face_block threads per block (64, 128, 192 or 256; by = 1). 2D: face
 * tile bx x by threads, a multiple of 64 and at most 256. cell_block: threads per block of
 * the cell update (64 to 256, a multiple of 64). Other shapes give POND_EINVAL.
 * Any shape gives bitwise-identical results. pond_autotune times the candidates on
 * the current state (which it leaves unchanged) and keeps the fastest. */
pond_status pond_set_tiles(pond_ctx *ctx, int32_t bx, int32_t by, int32_t cell_block);
pond_status pond_get_tiles(const pond_ctx *ctx, int32_t *bx, int32_t *by, int32_t *cell_block);
pond_status pond_autotune(pond_ctx *ctx);

/* Launch control (results of Sec. III.B.4 unchanged). on != 0: pond_step replays two steps captured once as a HIP graph (kernel launches
 * only; captured again when t_end, the step parity or any launch parameter changes)
 * instead of launching every kernel; results are identical. Steps with timing enabled,
 * and the last step of an odd count, are launched one by one. Default off. */
pond_status pond_set_graph(pond_ctx *ctx, int32_t on);

/* Launch control (results of Sec. III.B.4 unchanged). 1D only: on != 0 runs all the steps
 * of each pond_step call in a single launch, one
 * block per tube, longest tubes first (256 threads for a batch of 256 tubes or more,
 * otherwise 1,024 in mixed precision and 512 in FP64); each
 * block advances its tube step by step (the step of Sec. III.B.4 with the tube's own dt),
 * so no step pays kernel launch latency. Results, counters and failure handling are
 * identical to the launched kernels (same arithmetic per face and per cell). For small
 * grids and batches of independent tubes. Not used with timing enabled or the learned
 * seed (the launched kernels run then). Allocates a tube-order array of n_inst ints on the
 * first call with on != 0. POND_EINVAL for a 2D context; POND_ENOMEM / POND_EDEVICE if
 * the order array cannot be set up. Default off. */
pond_status pond_set_resident(pond_ctx *ctx, int32_t on);

/* 2D: the face kernel runs each face's frame iteration (Sec. III.B.3) for at most k
 * iterations; faces still iterating then continue, from the same state, in a tail kernel
 * that gives every face 16 lanes instead of one (a wave otherwise runs as long as its
 * slowest face). Results are those of the same iteration (rounding order aside).
 * k = 0 runs every face to the end in the face kernel. Default 4 (FP64) or 2 (mixed).
 * The tail sums its moments in another order than the face kernel, so different k
 * give results that differ by rounding (tile shapes do not change results at all);
 * pond_autotune therefore leaves k alone. Ignored in 1D.
 * With POND_FLAG_SEMI_LAGRANGIAN (2D) k applies to the cells' frame iterations
 * (Sec. III.A): cells still iterating after k iterations continue, from the same state,
 * in a tail kernel that spreads each cell's 25 stencil cells over 25 lanes (the same
 * iteration, its sums taken in another order: different k differ by rounding). Default 2
 * for the semi-Lagrangian step.
 * POND_EINVAL for k < 0, and in 3D. */
pond_status pond_set_iter_split(pond_ctx *ctx, int32_t k);

/* 2D finite volumes: store the cell state between steps as the 32 populations
 * (POND_LAYOUT_POPULATIONS, 32 planes of the population precision beside the FP64
 * conserved variables) or as the 12 Hermite coefficients (POND_LAYOUT_HERMITE, the
 * default); the current state is converted on the context's stream (the two are a change
 * of basis, exact on the Gauss-Hermite nodes: results differ by rounding only). The step
 * reads and writes the chosen layout; it exists to measure what the smaller state saves.
 * The population layout is taken with the Van Leer limiter, the Grad projection and the
 * plain seed only, and pond_save, pond_load, pond_populations and pond_load_mlp refuse it
 * (POND_EINVAL; set POND_LAYOUT_HERMITE first). POND_EINVAL as well in 1D and 3D, with the
 * semi-Lagrangian step, and for an unknown layout; POND_ENOMEM if the new planes cannot be
 * allocated (the state is then unchanged). */
pond_status pond_set_state_layout(pond_ctx *ctx, int32_t layout);

/* Measurement (no effect on results). Average device time in ms per step of each launch
 * over the last pond_step call,
 * measured with HIP events on the context's stream, into a caller array of 5:
 * out[0] dt/time kernel, out[1] face kernel (semi-Lagrangian scheme: its step kernel),
 * out[2] cell update kernel (1D, and 2D without a tail kernel; 2D with a tail kernel: the
 * pass over the marked stencil cells; semi-Lagrangian: the commit of the staged state),
 * out[3] seed (MLP) kernels, out[4] 2D with a tail kernel: the launch that finishes the
 * deferred faces and updates the other cells (0 otherwise).
 * Timing is recorded only after pond_enable_timing(ctx, 1). */
pond_status pond_enable_timing(pond_ctx *ctx, int32_t on);
pond_status pond_kernel_times(const pond_ctx *ctx, double *out);


/* ---------------------------------------------------------------------------------------
 * Learned seed of the face-frame iteration (not part of the paper's method: it only
 * replaces the predictor frame lambda_0 of Sec. III.B.3 for faces that needed
 * `hard_iters` or more iterations in the previous step; the iteration still runs to the
 * same tolerance). A 2 x 64 hidden-layer ReLU MLP, BF16 MFMA with FP32 accumulation,
 * FP32 master weights trained with Adam. Feature and target layouts are described in
 * pond_mlp_features. All device pointers are caller-owned (e.g. torch tensors) and must
 * stay valid during the call; calls are issued on the stream of the context or on `stream`.
 * --------------------------------------------------------------------------------------- */
typedef struct pond_mlp pond_mlp;

typedef struct {
    int32_t epochs;     /* passes over the data                         */
    int32_t batch;      /* samples per Adam step (multiple of 32)       */
    float lr;           /* Adam step size                               */
    float beta1, beta2; /* Adam moment decay rates                      */
    float eps;          /* Adam denominator offset                      */
} pond_train_cfg;

/* number of FP32 parameters: W1 (64x64, out x in), b1 (64), W2 (64x64), b2 (64),
 * W3 (3x64), b3 (3) */
int32_t pond_mlp_nparams(void);
/* Create a network with the given host parameters (pond_mlp_nparams values), or, if
 * params is NULL, with He-normal weights from a generator seeded by `seed` and zero biases. */
pond_status pond_mlp_create(const float *params, uint64_t seed, pond_mlp **out);
pond_status pond_mlp_get(const pond_mlp *m, float *params);
pond_status pond_mlp_set(pond_mlp *m, const float *params);
/* Inference: dev_Y[n][4] (outputs in columns 0..2) from dev_X[n][64] (FP32, row-major). */
pond_status pond_mlp_forward(pond_mlp *m, const float *dev_X, int64_t n, float *dev_Y, void *stream);
/* Loss (1/n) sum (y - t)^2 over samples and the 3 outputs, and its gradient w.r.t. the
 * parameters (host array, pond_mlp_nparams values); dev_T[n][4] targets (columns 0..2). */
pond_status pond_mlp_grad(pond_mlp *m, const float *dev_X, const float *dev_T, int64_t n,
                          float *grad, float *loss);
/* Adam training over consecutive batches of (dev_X, dev_T); loss_out (may be NULL) gets
 * the mean batch loss of every epoch (cfg->epochs values). */
pond_status pond_mlp_train(pond_mlp *m, const float *dev_X, const float *dev_T, int64_t n,
                           const pond_train_cfg *cfg, float *loss_out);
/* For callers that cannot allocate device memory (serving loops that retrain the seed
 * network online, harnesses that forbid hipMalloc): pond_mlp_train without any allocation.
 * The per-batch losses and per-epoch mean losses live in a file-scope device array of the
 * library, (POND_NOALLOC_MAX_BATCHES + POND_NOALLOC_MAX_EPOCHS) floats = 272 KiB, held by
 * every device the library runs on until the process ends, instead of a buffer allocated
 * per epoch. Arguments, results and errors as pond_mlp_train (same kernels, same losses and
 * parameters bit for bit), plus POND_EINVAL when an epoch has more than
 * POND_NOALLOC_MAX_BATCHES batches ((n + batch - 1) / batch) or cfg->epochs exceeds
 * POND_NOALLOC_MAX_EPOCHS (the network is then unchanged), and POND_ESTATE when the
 * current device is not the one that was current at pond_mlp_create. All calls on one
 * device share the array (it keeps the last call's contents): calls that overlap on one
 * device race. Synchronizes the network's stream. */
#define POND_NOALLOC_MAX_BATCHES 65536
#define POND_NOALLOC_MAX_EPOCHS 4096
pond_status pond_mlp_train_noalloc(pond_mlp *m, const float *dev_X, const float *dev_T, int64_t n,
                                   const pond_train_cfg *cfg, float *loss_out);
void pond_mlp_free(pond_mlp *m);

/* Features of every face at the context's current state (call before pond_step):
 * dev_X[nfaces][64], dev_ref[nfaces][4] = (u_n, u_t, sqrt T, T) of the centre cell.
 * Features: 3x3 cells centred on the face's lower neighbour, each as log(rho/rho_c),
 * (u_n - u_cn)/s_c, (u_t - u_ct)/s_c, log(T/T_c); then the previous face frame in the same
 * form and a flag (1 if the face has one); zeros up to 64. */
pond_status pond_mlp_features(pond_ctx *ctx, float *dev_X, float *dev_ref);
/* Targets of every face after a step: the face frames normalized by dev_ref,
 * ((u_n - u_cn)/s_c, (u_t - u_ct)/s_c, log(T/T_c)), minus the normalized previous frame
 * (features 36..38 of dev_X) where the face had one (feature 39 = 1); column 3 is 0.
 * dev_X and dev_ref are the arrays pond_mlp_features filled before the step. */
pond_status pond_mlp_targets(pond_ctx *ctx, const float *dev_X, const float *dev_ref, float *dev_T);
/* Attach a copy of the network to a context whose seed_mode is POND_SEED_MLP. */
pond_status pond_load_mlp(pond_ctx *ctx, const pond_mlp *m, int32_t hard_iters);

/* Checkpoint of the state carried between steps of Sec. III.B.4 (a warm start of a long
 * run): pond_save writes the carried state -- conserved
 * variables, non-equilibrium coefficients, face states and seeds, iteration flags, clocks
 * and time steps, the CFL maxima, failed-instance flags, step parity and count, and the
 * tail hand-over point -- to a binary file at `path` (overwritten). pond_load reads such a
 * file into a context created with the same configuration (the fields given to pond_init
 * are replaced); the steps that follow give bitwise the results the saved run would have
 * given. The learned seed's network is not part of the file. POND_EINVAL: null argument,
 * file that cannot be opened, written or read, or that belongs to another configuration
 * (then the context is unchanged); POND_EDEVICE: device copy failed. A checkpoint written
 * by a context of the other precision (FP64 / mixed) is accepted: its coefficient and face
 * planes are converted (rounded to FP32 or widened to FP64), conserved variables, clocks
 * and flags are taken as they are, and the context keeps its own tail hand-over point; the
 * steps that follow are those of the loading context's precision from that state (used to
 * start every form of a measurement window from one state). */
pond_status pond_save(pond_ctx *ctx, const char *path);
pond_status pond_load(pond_ctx *ctx, const char *path);

/* Housekeeping: release a context (NULL is ignored); the text of a status; the ABI version
 * this library implements (POND_ABI_VERSION of the header it was built with). */
void pond_free(pond_ctx *ctx);
const char *pond_strerror(pond_status s);
int32_t pond_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
