// pond.hip -- host side of libpond: the C ABI of include/pond.h on top of the kernels in
// pond_kernels.hpp. The library owns its device memory (hipMalloc) and issues all work on
// one stream per context; nothing here computes the method, it only validates, allocates,
// launches and copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pond.h"
#include "pond_kernels.hpp"
#include "pond_kernels3d.hpp"
#include "pond_sl2d.hpp"
#include "pond_mlp.hpp"

using namespace pond;

struct pond_ctx {
    pond_config cfg;
    Params P;
    int D;
    int precision;
    int nh, nfp; // planes of H and F
    int layout = POND_LAYOUT_HERMITE; // 2D: the state as coefficients (H) or populations
    size_t rsize;
    hipStream_t stream;
    hipStream_t own_stream;
    // device buffers
    double *U = nullptr;
    void *H = nullptr, *F = nullptr;
    int *fiter = nullptr;
    int *cell_inst = nullptr, *face_inst = nullptr;
    int64_t *cell_off = nullptr, *pad_off = nullptr;
    double *t = nullptr, *tstart = nullptr, *dt = nullptr, *dxk = nullptr;
    unsigned long long *vmax = nullptr, *stats = nullptr;
    int *err = nullptr;
    int *inst_err = nullptr;
    double *scratch = nullptr; // read-out staging (4 x max(ncell, nface) doubles) and summary records
    // 2D: faces handed from the face kernel to the tail kernel
    int *tail_f = nullptr, *tail_meta = nullptr, *tail_count = nullptr, *tblock = nullptr;
    void *tail_s = nullptr;
    // host mirrors
    std::vector<int64_t> h_cell_off;
    std::vector<int> h_failed; // failed-instance flags at the end of the last pond_step call
    int tube_span = 0;
    int slot = 0;
    int64_t steps_done = 0;
    // launch shapes
    int bx = 256, by = 1, cell_block = 256;
    // timing: one set of 6 events per step of a pond_step call, read once at its end
    int timing = 0;
    double ktime[5] = {0, 0, 0, 0, 0};
    std::vector<hipEvent_t> evs;
    hipEvent_t *ev = nullptr;
    // learned seed
    MlpDevice mlp;
    // optional replay of two captured steps (hipGraph); invalid after any change of launch
    // parameters
    int use_graph = 0;
    hipGraphExec_t gexec = nullptr;
    double g_tend = 0.0;
    int g_slot = -1;
    // 1D: every step of a pond_step call in one launch, one block per tube (longest first)
    int resident = 0;
    // semi-Lagrangian scheme: staging of the new state, and the largest number of tube
    // boundaries inside a block of 256 cells
    double *U2 = nullptr;
    void *H2 = nullptr;
    int sl_span = 0;
    int *res_order = nullptr;
    // 3D: geometry, and the phi-bar-plus records of the cells (NR3 planes, precision R)
    Geo3 G3;
    void *rec3 = nullptr;
};

static void drop_graph(pond_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
}

namespace {

const char *kErr[] = {"ok", "invalid argument", "device allocation failed", "HIP runtime error",
                      "face iteration did not converge", "departure point outside upwind cell",
                      "non-physical cell state", "invalid call for the context state"};

bool hip_ok(hipError_t e)
{
    if (e != hipSuccess) {
        fprintf(stderr, "libpond: HIP error %s\n", hipGetErrorString(e));
        return false;
    }
    return true;
}

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        if (!hip_ok(x)) return POND_EDEVICE;                                                       \
    } while (0)

template <typename R>
State<R> state_of(pond_ctx *c)
{
    State<R> S;
    S.U = c->U;
    S.H = reinterpret_cast<R *>(c->H);
    S.F = reinterpret_cast<R *>(c->F);
    S.fiter = c->fiter;
    S.cell_inst = c->cell_inst;
    S.face_inst = c->face_inst;
    S.cell_off = c->cell_off;
    S.pad_off = c->pad_off;
    S.t = c->t;
    S.tstart = c->tstart;
    S.dt = c->dt;
    S.dxk = c->dxk;
    S.vmax = c->vmax;
    S.stats = c->stats;
    S.err = c->err;
    S.inst_err = c->inst_err;
    S.U2 = c->U2;
    S.H2 = reinterpret_cast<R *>(c->H2);
    S.tail_f = c->tail_f;
    S.tail_s = reinterpret_cast<R *>(c->tail_s);
    S.tail_meta = c->tail_meta;
    S.tail_count = c->tail_count;
    S.tblock = c->tblock;
    S.seed_count = (c->cfg.seed_mode == POND_SEED_MLP && c->mlp.ready) ? c->mlp.count : nullptr;
    return S;
}

unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// 2D face tiles the autotuner tries (the first is the default)
const std::pair<int, int> kTiles2D[] = {{8, 8}, {16, 4}, {16, 8}, {16, 16}, {32, 8}, {64, 4}, {32, 2}};

// entries one sub-list of the tail list must hold for a face launch with bx x by tiles: the
// waves of its slot (the global wave index modulo NSLOT) times 64 faces of one axis
int64_t tail_cap_for(const pond_ctx *c, int bx, int by)
{
    const int64_t nb = (int64_t)blocks(c->P.nx + 1, bx) * blocks(c->P.ny + 1, by);
    const int64_t waves = nb * ((bx * by + 63) / 64);
    return 64 * ((waves + NSLOT - 1) / NSLOT);
}

// grow the tail list for a launch shape that needs more room (between steps)
bool ensure_tail(pond_ctx *c, int bx, int by)
{
    const int64_t need = tail_cap_for(c, bx, by);
    if (need <= c->P.tail_cap) return true;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return false;
    const int64_t n = 2 * NSLOT * need;
    int *f = nullptr, *m = nullptr;
    void *st = nullptr;
    if (hipMalloc(&f, sizeof(int) * n) != hipSuccess || hipMalloc(&m, sizeof(int) * n) != hipSuccess ||
        hipMalloc(&st, c->rsize * 6 * n) != hipSuccess) {
        (void)hipFree(f);
        (void)hipFree(m);
        (void)hipFree(st);
        return false;
    }
    (void)hipFree(c->tail_f);
    (void)hipFree(c->tail_meta);
    (void)hipFree(c->tail_s);
    c->tail_f = f;
    c->tail_meta = m;
    c->tail_s = st;
    c->P.tail_cap = (int)need;
    c->P.tail_n = n;
    return true;
}

// plane stride of the 2D face kernel's LDS tile: 256 or 512 (compiled in), else the tile's
// own size
// LDS plane stride of the 2D face kernel's record tile (a compile-time constant, so that every
// record load takes its plane offset as an immediate): the smallest of 256, 384 (FP64 only)
// and 512 that holds the tile's records, else 0 (a run-time stride). The byte offset of a
// plane must fit the LDS instruction's 16-bit offset field: 18 planes of 512 doubles do not
// (the last two planes then need an address register, and the FP64 kernel spills), 18 of 384
// do, and a 16 x 16 tile needs 361 records.
int face_nts(int bx, int by, size_t rsize)
{
    const int n = (bx + 3) * (by + 3);
    if (n <= 256) return 256;
    if (rsize == 8 && n <= 384) return 384;
    return n <= 512 ? 512 : 0;
}

size_t face_lds_bytes(const pond_ctx *c, int bx, int by, int span)
{
    if (c->D == 1) return (size_t)(bx + 3 + 3 * span) * Layout<1>::NL * c->rsize;
    const int nts = face_nts(bx, by, c->rsize);
    return (size_t)(nts ? nts : (bx + 3) * (by + 3)) * Layout<2>::NL * c->rsize;
}

// 1: the alternative regularization of the f populations (2D only; in 1D it changes nothing)
int reg_of(const pond_ctx *c) { return (c->D == 2 && (c->cfg.flags & POND_FLAG_REG_EQ)) ? 1 : 0; }

template <typename R, int LIM, int REG, int LAY = 0>
void launch_face_2d_reg(pond_ctx *c, const State<R> &S, int bx, int by, size_t lds)
{
    dim3 grid(blocks(c->P.nx + 1, bx), blocks(c->P.ny + 1, by));
    switch (face_nts(bx, by, sizeof(R))) {
    case 256:
        face_kernel_2d<R, LIM, 256, REG, LAY><<<grid, dim3(bx, by), lds, c->stream>>>(c->P, S);
        break;
    case 384:
        if constexpr (sizeof(R) == 8)
            face_kernel_2d<R, LIM, 384, REG, LAY><<<grid, dim3(bx, by), lds, c->stream>>>(c->P, S);
        break;
    case 512:
        face_kernel_2d<R, LIM, 512, REG, LAY><<<grid, dim3(bx, by), lds, c->stream>>>(c->P, S);
        break;
    default:
        face_kernel_2d<R, LIM, 0, REG, LAY><<<grid, dim3(bx, by), lds, c->stream>>>(c->P, S);
    }
}

// (the population layout is taken with the Van Leer limiter and the Grad projection only)
template <typename R, int LIM>
void launch_face_2d(pond_ctx *c, const State<R> &S, int bx, int by, size_t lds)
{
    if (c->layout == POND_LAYOUT_POPULATIONS)
        launch_face_2d_reg<R, 0, 0, 1>(c, S, bx, by, lds);
    else if (reg_of(c))
        launch_face_2d_reg<R, LIM, 1>(c, S, bx, by, lds);
    else
        launch_face_2d_reg<R, LIM, 0>(c, S, bx, by, lds);
}

template <typename R, int REG>
void launch_face_tail_reg(pond_ctx *c, const State<R> &S)
{
    // per axis, 1,024 blocks of 16 faces take the deferred faces in turn
    dim3 tgrid(NSLOT * 4, 2);
    if (c->layout == POND_LAYOUT_POPULATIONS)
        face_tail_kernel_2d<R, 0, 0, 1><<<tgrid, 256, 0, c->stream>>>(c->P, S);
    else if (c->P.limiter == POND_LIM_MINMOD)
        face_tail_kernel_2d<R, 1, REG><<<tgrid, 256, 0, c->stream>>>(c->P, S);
    else
        face_tail_kernel_2d<R, 0, REG><<<tgrid, 256, 0, c->stream>>>(c->P, S);
}

// the tail beside the update of the cells outside its faces' stencils, then those
template <typename R, int REG>
void launch_tail_cells_reg(pond_ctx *c, const State<R> &S, hipEvent_t ev_mid)
{
    const unsigned nb = 2 * TAIL_BLOCKS + (unsigned)blocks(c->P.ncell, 256);
    const bool pops = c->layout == POND_LAYOUT_POPULATIONS;
    if (pops)
        tail_cell_kernel_2d<R, 0, 0, 1><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
    else if (c->P.limiter == POND_LIM_MINMOD)
        tail_cell_kernel_2d<R, 1, REG><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
    else
        tail_cell_kernel_2d<R, 0, REG><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
    if (ev_mid) (void)hipEventRecord(ev_mid, c->stream);
    if (pops)
        cell_marked_kernel_2d<R, 0, 1><<<blocks(c->P.ncell, 256), 256, 0, c->stream>>>(c->P, S, c->slot);
    else
        cell_marked_kernel_2d<R, REG><<<blocks(c->P.ncell, 256), 256, 0, c->stream>>>(c->P, S, c->slot);
}

int compute_span(const pond_ctx *c, int B)
{
    // largest number of tube boundaries inside one block of B faces
    if (c->cfg.dim != 1 || c->P.n_inst == 1) return 0;
    int64_t nf = c->P.nface;
    int span = 0;
    const auto &off = c->h_cell_off;
    int k = 0;
    for (int64_t f0 = 0; f0 < nf; f0 += B) {
        int64_t fl = std::min(f0 + B, nf) - 1;
        while (k + 1 < c->P.n_inst && off[k + 1] + (k + 1) <= f0) ++k;
        int k1 = k;
        while (k1 + 1 < c->P.n_inst && off[k1 + 1] + (k1 + 1) <= fl) ++k1;
        span = std::max(span, k1 - k);
    }
    return span;
}

// largest number of tube boundaries inside one block of B cells
int compute_cell_span(const pond_ctx *c, int B)
{
    if (c->cfg.dim != 1 || c->P.n_inst == 1) return 0;
    const int64_t n = c->P.ncell;
    const auto &off = c->h_cell_off;
    int span = 0, k = 0;
    for (int64_t c0 = 0; c0 < n; c0 += B) {
        const int64_t cl = std::min(c0 + B, n) - 1;
        while (k + 1 < c->P.n_inst && off[k + 1] <= c0) ++k;
        int k1 = k;
        while (k1 + 1 < c->P.n_inst && off[k1 + 1] <= cl) ++k1;
        span = std::max(span, k1 - k);
    }
    return span;
}

bool semi_lagrangian(const pond_ctx *c) { return (c->cfg.flags & POND_FLAG_SEMI_LAGRANGIAN) != 0; }

// the face kernel, and in 2D (with_tail) the tail kernel after it
template <int D, typename R>
hipError_t launch_face(pond_ctx *c, int bx, int by, bool with_tail)
{
    State<R> S = state_of<R>(c);
    if (D == 1) {
        int span = (bx == c->bx) ? c->tube_span : compute_span(c, bx);
        size_t lds = face_lds_bytes(c, bx, 1, span);
        if (c->P.limiter == POND_LIM_MINMOD)
            face_kernel_1d<R, 1><<<blocks(c->P.nface, bx), bx, lds, c->stream>>>(c->P, S, span);
        else
            face_kernel_1d<R, 0><<<blocks(c->P.nface, bx), bx, lds, c->stream>>>(c->P, S, span);
    } else {
        size_t lds = face_lds_bytes(c, bx, by, 0);
        if (c->P.limiter == POND_LIM_MINMOD)
            launch_face_2d<R, 1>(c, S, bx, by, lds);
        else
            launch_face_2d<R, 0>(c, S, bx, by, lds);
        if (with_tail && c->P.iter_split > 0) {
            if (reg_of(c))
                launch_face_tail_reg<R, 1>(c, S);
            else
                launch_face_tail_reg<R, 0>(c, S);
        }
    }
    return hipGetLastError();
}

template <int D, typename R>
hipError_t launch_step(pond_ctx *c, double t_end)
{
    State<R> S = state_of<R>(c);
    const bool tm = c->ev != nullptr;
    if (tm) (void)hipEventRecord(c->ev[0], c->stream);
    dt_kernel<D, R><<<c->P.n_inst, 64, 0, c->stream>>>(c->P, S, t_end, c->slot);
    if (tm) (void)hipEventRecord(c->ev[1], c->stream);
    if (c->cfg.seed_mode == POND_SEED_MLP && c->mlp.ready) {
        hipError_t e = mlp_seed_launch<D, R>(c->mlp, c->P, S, c->stream);
        if (e != hipSuccess) return e;
    }
    if (tm) (void)hipEventRecord(c->ev[2], c->stream);
    if (semi_lagrangian(c)) {
        // semi-Lagrangian step: every cell into the staging buffers, then committed
        if (D == 1) {
            const size_t lds = (size_t)(256 + 4 + 4 * c->sl_span) * Layout<1>::NL * sizeof(R);
            sl_kernel_1d<R><<<blocks(c->P.ncell, 256), 256, lds, c->stream>>>(c->P, S, c->sl_span, c->slot);
        } else {
            // cells still iterating after iter_split iterations are finished by the tail kernel
            const int nb = ((c->P.nx + SL2_T - 1) / SL2_T) * ((c->P.ny + SL2_T - 1) / SL2_T);
            const bool split = c->P.iter_split > 0;
            if (reg_of(c)) {
                if (split)
                    sl_kernel_2d<R, 1, true><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
                else
                    sl_kernel_2d<R, 1, false><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
            } else {
                if (split)
                    sl_kernel_2d<R, 0, true><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
                else
                    sl_kernel_2d<R, 0, false><<<nb, 256, 0, c->stream>>>(c->P, S, c->slot);
            }
            if (tm) (void)hipEventRecord(c->ev[3], c->stream);
            if (split) {
                if (reg_of(c))
                    sl_tail_kernel_2d<R, 1><<<SL2_TAIL_BLOCKS, 64, 0, c->stream>>>(c->P, S, c->slot);
                else
                    sl_tail_kernel_2d<R, 0><<<SL2_TAIL_BLOCKS, 64, 0, c->stream>>>(c->P, S, c->slot);
            }
        }
        if (tm && D == 1) (void)hipEventRecord(c->ev[3], c->stream);
        if (tm) (void)hipEventRecord(c->ev[4], c->stream);
        sl_commit_kernel<R><<<blocks(c->P.ncell, 256), 256, 0, c->stream>>>(c->P, S, c->nh);
        if (tm) (void)hipEventRecord(c->ev[5], c->stream);
        c->slot ^= 1;
        return hipGetLastError();
    }
    hipError_t e = launch_face<D, R>(c, c->bx, c->by, false);
    if (e != hipSuccess) return e;
    if (tm) (void)hipEventRecord(c->ev[3], c->stream);
    if (D == 2 && c->P.iter_split > 0) {
        if (reg_of(c))
            launch_tail_cells_reg<R, 1>(c, S, tm ? c->ev[4] : nullptr);
        else
            launch_tail_cells_reg<R, 0>(c, S, tm ? c->ev[4] : nullptr);
    } else {
        if (tm) (void)hipEventRecord(c->ev[4], c->stream);
        if (D == 2 && c->layout == POND_LAYOUT_POPULATIONS)
            cell_kernel<2, R, 0, 1><<<blocks(c->P.ncell, c->cell_block), c->cell_block, 0, c->stream>>>(c->P, S, c->slot);
        else if (reg_of(c))
            cell_kernel<D, R, 1><<<blocks(c->P.ncell, c->cell_block), c->cell_block, 0, c->stream>>>(c->P, S, c->slot);
        else
            cell_kernel<D, R, 0><<<blocks(c->P.ncell, c->cell_block), c->cell_block, 0, c->stream>>>(c->P, S, c->slot);
    }
    if (tm) (void)hipEventRecord(c->ev[5], c->stream);
    c->slot ^= 1;
    return hipGetLastError();
}

// the resident 1D kernel. Fewer tubes than compute units: the largest block that the face
// code fits, so that one tube spreads over as many lanes as it can (1,024 threads in mixed
// precision, where the FP32 face code fits the 128 registers that leaves; 512 in FP64).
// A batch of at least as many tubes as compute units: 256-thread blocks, several per
// compute unit, whose tubes hide each other's latencies (4096 tubes of 200-4,000 cells:
// 0.28 against 0.37 ms per step in mixed precision, 0.53 against 0.71 in FP64).
template <typename R, int NT>
void launch_resident_nt(pond_ctx *c, const State<R> &S, int nsteps, double t_end)
{
    const size_t lds = (size_t)(NT + 3) * Layout<1>::NL * sizeof(R);
    if (c->P.limiter == POND_LIM_MINMOD)
        tube_resident_kernel_1d<R, 1, NT><<<c->P.n_inst, NT, lds, c->stream>>>(c->P, S, t_end, nsteps, c->slot,
                                                                                 c->res_order);
    else
        tube_resident_kernel_1d<R, 0, NT><<<c->P.n_inst, NT, lds, c->stream>>>(c->P, S, t_end, nsteps, c->slot,
                                                                                 c->res_order);
}

constexpr int RESIDENT_BATCH = 256; // compute units of the MI355X

template <typename R>
hipError_t launch_resident(pond_ctx *c, int nsteps, double t_end)
{
    State<R> S = state_of<R>(c);
    if (c->P.n_inst >= RESIDENT_BATCH)
        launch_resident_nt<R, 256>(c, S, nsteps, t_end);
    else
        launch_resident_nt<R, sizeof(R) == 8 ? 512 : 1024>(c, S, nsteps, t_end);
    c->slot ^= nsteps & 1;
    return hipGetLastError();
}

// 3D: dt, the phi-bar-plus records, the faces of each axis, the cells
template <typename R>
hipError_t launch_step3(pond_ctx *c, double t_end)
{
    State<R> S = state_of<R>(c);
    R *rec = reinterpret_cast<R *>(c->rec3);
    const bool tm = c->ev != nullptr;
    if (tm) (void)hipEventRecord(c->ev[0], c->stream);
    dt_kernel<3, R><<<1, 64, 0, c->stream>>>(c->P, S, t_end, c->slot);
    if (tm) (void)hipEventRecord(c->ev[1], c->stream);
    if (tm) (void)hipEventRecord(c->ev[2], c->stream);
    plus_kernel_3d<R><<<blocks(c->P.ncell, 256), 256, 0, c->stream>>>(c->P, S, rec);
    const Geo3 &G = c->G3;
    const bool mm = c->P.limiter == POND_LIM_MINMOD;
    // one block per 64 faces of a row of faces along x (the stencil rows staged in LDS)
    constexpr int FPB = fpb3<R>(), NTH = 4 * FPB;
    const unsigned b0 = (unsigned)face3_blocks(G, 0, FPB), b1 = (unsigned)face3_blocks(G, 1, FPB),
                   b2 = (unsigned)face3_blocks(G, 2, FPB);
    if (mm) {
        face_kernel_3d<R, 0, 1><<<b0, NTH, 0, c->stream>>>(c->P, G, S, rec);
        face_kernel_3d<R, 1, 1><<<b1, NTH, 0, c->stream>>>(c->P, G, S, rec);
        face_kernel_3d<R, 2, 1><<<b2, NTH, 0, c->stream>>>(c->P, G, S, rec);
    } else {
        face_kernel_3d<R, 0, 0><<<b0, NTH, 0, c->stream>>>(c->P, G, S, rec);
        face_kernel_3d<R, 1, 0><<<b1, NTH, 0, c->stream>>>(c->P, G, S, rec);
        face_kernel_3d<R, 2, 0><<<b2, NTH, 0, c->stream>>>(c->P, G, S, rec);
    }
    if (tm) (void)hipEventRecord(c->ev[3], c->stream);
    if (tm) (void)hipEventRecord(c->ev[4], c->stream);
    cell_kernel_3d<R><<<blocks(c->P.ncell, 256), 256, 0, c->stream>>>(c->P, G, S, c->slot);
    if (tm) (void)hipEventRecord(c->ev[5], c->stream);
    c->slot ^= 1;
    return hipGetLastError();
}

hipError_t step_once(pond_ctx *c, double t_end)
{
    if (c->D == 3)
        return c->precision == POND_FP64 ? launch_step3<double>(c, t_end) : launch_step3<float>(c, t_end);
    if (c->D == 1)
        return c->precision == POND_FP64 ? launch_step<1, double>(c, t_end) : launch_step<1, float>(c, t_end);
    return c->precision == POND_FP64 ? launch_step<2, double>(c, t_end) : launch_step<2, float>(c, t_end);
}

hipError_t face_once(pond_ctx *c, int bx, int by)
{
    if (c->tail_count) tail_reset_kernel<<<1, 64, 0, c->stream>>>(c->tail_count);
    if (c->D == 1)
        return c->precision == POND_FP64 ? launch_face<1, double>(c, bx, by, true)
                                         : launch_face<1, float>(c, bx, by, true);
    hipError_t e = c->precision == POND_FP64 ? launch_face<2, double>(c, bx, by, true)
                                             : launch_face<2, float>(c, bx, by, true);
    // no cell update follows here: clear the stencil marks the face kernel set
    if (e == hipSuccess && c->tblock) {
        clear_ints_kernel<<<blocks(c->P.ncell, 256), 256, 0, c->stream>>>(c->tblock, c->P.ncell);
        e = hipGetLastError();
    }
    return e;
}

// 3D: sizes, extents, the three boundary kinds, what the 3D path does not take
pond_status validate3(const pond_config *cfg, const double *rho, const double *ux, const double *uy,
                      const double *uz, const double *p)
{
    if (!uy || !uz || cfg->nx < 2 || cfg->ny < 2 || cfg->nz < 2) return POND_EINVAL;
    if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0 && cfg->cfl < 1.0) || !(cfg->mu > 0.0)) return POND_EINVAL;
    if (!(cfg->tol > 0.0) || cfg->max_iter < 1 || cfg->max_iter > 60000) return POND_EINVAL;
    if (!(cfg->x1 > cfg->x0) || !(cfg->y1 > cfg->y0) || !(cfg->z1 > cfg->z0)) return POND_EINVAL;
    if (cfg->precision != POND_FP64 && cfg->precision != POND_MIXED) return POND_EINVAL;
    if (cfg->limiter != POND_LIM_VANLEER && cfg->limiter != POND_LIM_MINMOD) return POND_EINVAL;
    if (cfg->flags & ~POND_FLAG_STRICT) return POND_EINVAL;
    if (cfg->seed_mode != POND_SEED_PREV) return POND_EINVAL;
    if (!(1.0 / (cfg->gamma - 1.0) - 1.5 >= 0.0)) return POND_EINVAL;
    int kinds[6] = {cfg->bc[0], cfg->bc[1], cfg->bc[2], cfg->bc[3], cfg->bc_z[0], cfg->bc_z[1]};
    for (int s = 0; s < 6; ++s)
        if (kinds[s] != POND_BC_PERIODIC && kinds[s] != POND_BC_OUTFLOW && kinds[s] != POND_BC_REFLECT)
            return POND_EINVAL;
    for (int a = 0; a < 3; ++a)
        if ((kinds[2 * a] == POND_BC_PERIODIC) != (kinds[2 * a + 1] == POND_BC_PERIODIC)) return POND_EINVAL;
    const int64_t n = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    if (n > (int64_t)INT32_MAX / 4) return POND_EINVAL; // cell indices are 32-bit in the kernels
    for (int64_t i = 0; i < n; ++i)
        if (!(rho[i] > 0.0) || !(p[i] > 0.0) || !std::isfinite(rho[i]) || !std::isfinite(p[i]) ||
            !std::isfinite(ux[i]) || !std::isfinite(uy[i]) || !std::isfinite(uz[i]))
            return POND_EINVAL;
    return POND_OK;
}

pond_status validate(const pond_config *cfg, const double *rho, const double *ux, const double *uy,
                     const double *p)
{
    if (!cfg || !rho || !ux || !p) return POND_EINVAL;
    if (cfg->dim != 1 && cfg->dim != 2) return POND_EINVAL;
    if (cfg->dim == 2 && (!uy || cfg->nx < 2 || cfg->ny < 2)) return POND_EINVAL;
    if (cfg->dim == 1 && (cfg->n_inst < 1 || (cfg->n_inst > 1 && !cfg->len))) return POND_EINVAL;
    if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0 && cfg->cfl < 1.0) || !(cfg->mu > 0.0)) return POND_EINVAL;
    if (!(cfg->tol > 0.0) || cfg->max_iter < 1 || cfg->max_iter > 60000) return POND_EINVAL;
    if (!(cfg->x1 > cfg->x0) || (cfg->dim == 2 && !(cfg->y1 > cfg->y0))) return POND_EINVAL;
    if (cfg->precision != POND_FP64 && cfg->precision != POND_MIXED) return POND_EINVAL;
    if (cfg->limiter != POND_LIM_VANLEER && cfg->limiter != POND_LIM_MINMOD) return POND_EINVAL;
    if (cfg->flags & ~(POND_FLAG_STRICT | POND_FLAG_REG_EQ | POND_FLAG_SEMI_LAGRANGIAN)) return POND_EINVAL;
    if ((cfg->flags & POND_FLAG_SEMI_LAGRANGIAN) && (cfg->dim > 2 || cfg->seed_mode != POND_SEED_PREV))
        return POND_EINVAL;
    double Cv = 1.0 / (cfg->gamma - 1.0);
    if (!(Cv - 0.5 * cfg->dim > 0.0)) return POND_EINVAL;
    for (int s = 0; s < 4; ++s) {
        int b = cfg->bc[s];
        if (b < POND_BC_PERIODIC || b > POND_BC_MOVING_SHOCK) return POND_EINVAL;
        if (cfg->dim == 1 && s >= 2) continue;
        if (b == POND_BC_FIXED || b == POND_BC_FIXED_WINDOW || b == POND_BC_SPLIT_FIXED_REFLECT ||
            b == POND_BC_MOVING_SHOCK) {
            if (!(cfg->bc_state[s][0] > 0.0) || !(cfg->bc_state[s][3] > 0.0)) return POND_EINVAL;
        }
        if ((b == POND_BC_FIXED_WINDOW || b == POND_BC_MOVING_SHOCK) &&
            (!(cfg->bc_alt[s][0] > 0.0) || !(cfg->bc_alt[s][3] > 0.0)))
            return POND_EINVAL;
    }
    // periodic sides come in pairs
    if ((cfg->bc[0] == POND_BC_PERIODIC) != (cfg->bc[1] == POND_BC_PERIODIC)) return POND_EINVAL;
    if (cfg->dim == 2 && (cfg->bc[2] == POND_BC_PERIODIC) != (cfg->bc[3] == POND_BC_PERIODIC))
        return POND_EINVAL;
    int64_t n = 0;
    if (cfg->dim == 1) {
        if (cfg->n_inst == 1 && !cfg->len) {
            if (cfg->nx < 4) return POND_EINVAL;
            n = cfg->nx;
        } else {
            for (int k = 0; k < cfg->n_inst; ++k) {
                if (cfg->len[k] < 4) return POND_EINVAL;
                n += cfg->len[k];
            }
            if (n != cfg->nx) return POND_EINVAL;
            if (cfg->n_inst > 1 && (cfg->bc[0] == POND_BC_PERIODIC)) return POND_EINVAL;
        }
    } else {
        n = (int64_t)cfg->nx * cfg->ny;
    }
    for (int64_t i = 0; i < n; ++i) {
        if (!(rho[i] > 0.0) || !(p[i] > 0.0) || !std::isfinite(rho[i]) || !std::isfinite(p[i]) ||
            !std::isfinite(ux[i]) || (cfg->dim == 2 && !std::isfinite(uy[i])))
            return POND_EINVAL;
    }
    return POND_OK;
}

template <int D, typename R>
void init_launch(pond_ctx *c, const double *dprim)
{
    State<R> S = state_of<R>(c);
    int64_t nmax = std::max(c->P.ncell, c->P.nface);
    init_kernel<D, R><<<blocks(nmax, 256), 256, 0, c->stream>>>(c->P, S, dprim, c->nh);
}

void free_all(pond_ctx *c)
{
    void *ptrs[] = {c->U, c->H, c->F, c->fiter, c->cell_inst, c->face_inst, c->cell_off, c->pad_off,
                    c->t, c->tstart, c->dt, c->dxk, c->vmax, c->stats, c->err, c->inst_err, c->scratch,
                    c->tail_f, c->tail_s, c->tail_meta, c->tail_count, c->tblock, c->res_order,
                    c->U2, c->H2, c->rec3};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    mlp_free(c->mlp);
}

} // namespace

extern "C" {

int32_t pond_abi_version(void) { return POND_ABI_VERSION; }

const char *pond_strerror(pond_status s)
{
    if ((int)s < 0 || (int)s > 7) return "unknown status";
    return kErr[(int)s];
}

pond_status pond_init(const pond_config *cfg, const double *rho, const double *ux, const double *uy,
                      const double *p, pond_ctx **out)
{
    if (!out) return POND_EINVAL;
    *out = nullptr;
    if (cfg && cfg->dim == 3) return POND_EINVAL; // needs the z velocity: pond_init3
    return pond_init3(cfg, rho, ux, uy, nullptr, p, out);
}

pond_status pond_init3(const pond_config *cfg, const double *rho, const double *ux, const double *uy,
                       const double *uz, const double *p, pond_ctx **out)
{
    if (!out) return POND_EINVAL;
    *out = nullptr;
    if (!cfg || !rho || !ux || !p) return POND_EINVAL;
    pond_status v = (cfg->dim == 3) ? validate3(cfg, rho, ux, uy, uz, p) : validate(cfg, rho, ux, uy, p);
    if (v != POND_OK) return v;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return POND_EDEVICE;
    pond_ctx *c = new (std::nothrow) pond_ctx();
    if (!c) return POND_ENOMEM;
    c->cfg = *cfg;
    c->cfg.len = nullptr;
    c->D = cfg->dim;
    c->precision = cfg->precision;
    c->rsize = (cfg->precision == POND_FP64) ? sizeof(double) : sizeof(float);
    Params &P = c->P;
    memset(&P, 0, sizeof(P));
    P.dim = cfg->dim;
    P.nx = cfg->nx;
    P.ny = (cfg->dim >= 2) ? cfg->ny : 1;
    P.n_inst = (cfg->dim == 1) ? cfg->n_inst : 1;
    P.x0 = cfg->x0;
    P.y0 = cfg->y0;
    P.Cv = 1.0 / (cfg->gamma - 1.0);
    P.cfl = cfg->cfl;
    P.mu = cfg->mu;
    P.tol = cfg->tol;
    P.limiter = cfg->limiter;
    P.max_iter = cfg->max_iter;
    for (int s = 0; s < 4; ++s) {
        P.bc[s] = cfg->bc[s];
        for (int q = 0; q < 4; ++q) {
            P.bc_state[s][q] = cfg->bc_state[s][q];
            P.bc_alt[s][q] = cfg->bc_alt[s][q];
            P.bc_param[s][q] = cfg->bc_param[s][q];
        }
    }
    // fastest particle speed, per axis, of the states the boundary conditions prescribe
    for (int s = 0; s < 2 * std::min(cfg->dim, 2); ++s) {
        const double *used[2] = {nullptr, nullptr};
        if (P.bc[s] == BC_FIXED || P.bc[s] == BC_SPLIT) used[0] = cfg->bc_state[s];
        if (P.bc[s] == BC_FIXED_WINDOW || P.bc[s] == BC_MOVING) {
            used[0] = cfg->bc_state[s];
            used[1] = cfg->bc_alt[s];
        }
        for (const double *st : used) {
            if (!st) continue;
            double T = st[3] / st[0];
            for (int a = 0; a < cfg->dim; ++a)
                P.bc_speed[a] = std::max(P.bc_speed[a], std::fabs(st[1 + a]) + std::sqrt(T) * CMAX);
        }
    }
    // per-instance layout (1D tubes concatenated; each tube spans [x0, x1])
    std::vector<int64_t> coff(P.n_inst + 1, 0), poff(P.n_inst + 1, 0);
    std::vector<int> len(P.n_inst);
    for (int k = 0; k < P.n_inst; ++k) len[k] = (cfg->dim == 1 && cfg->len) ? cfg->len[k] : cfg->nx;
    for (int k = 0; k < P.n_inst; ++k) coff[k + 1] = coff[k] + len[k];
    for (int k = 0; k <= P.n_inst; ++k) poff[k] = coff[k] + 4 * (int64_t)k;
    c->h_cell_off = coff;
    if (cfg->dim == 1) {
        P.ncell = coff[P.n_inst];
        P.nface = P.ncell + P.n_inst;
        P.nfx = P.nface;
        // every tube spans [x0, x1]: its own cell size is kept per instance
        P.dx = (cfg->x1 - cfg->x0) / len[0];
        P.dy = 1.0;
    } else if (cfg->dim == 2) {
        P.ncell = (int64_t)P.nx * P.ny;
        P.nfx = (int64_t)(P.nx + 1) * P.ny;
        P.nface = P.nfx + (int64_t)P.nx * (P.ny + 1);
        P.dx = (cfg->x1 - cfg->x0) / P.nx;
        P.dy = (cfg->y1 - cfg->y0) / P.ny;
    } else {
        Geo3 &G = c->G3;
        G.nx = cfg->nx;
        G.ny = cfg->ny;
        G.nz = cfg->nz;
        G.dx[0] = (cfg->x1 - cfg->x0) / cfg->nx;
        G.dx[1] = (cfg->y1 - cfg->y0) / cfg->ny;
        G.dx[2] = (cfg->z1 - cfg->z0) / cfg->nz;
        const int kinds[6] = {cfg->bc[0], cfg->bc[1], cfg->bc[2], cfg->bc[3], cfg->bc_z[0], cfg->bc_z[1]};
        for (int q = 0; q < 6; ++q) G.bc[q] = kinds[q];
        G.nfa[0] = (int64_t)(G.nx + 1) * G.ny * G.nz;
        G.nfa[1] = (int64_t)G.nx * (G.ny + 1) * G.nz;
        G.nfa[2] = (int64_t)G.nx * G.ny * (G.nz + 1);
        G.foff[0] = 0;
        G.foff[1] = G.nfa[0];
        G.foff[2] = G.nfa[0] + G.nfa[1];
        P.ncell = (int64_t)G.nx * G.ny * G.nz;
        P.nfx = G.nfa[0];
        P.nface = G.nfa[0] + G.nfa[1] + G.nfa[2];
        P.dx = G.dx[0];
        P.dy = G.dx[1];
    }
    c->nh = (c->D == 1) ? Layout<1>::NH : (c->D == 2) ? Layout<2>::NH : NH3;
    c->nfp = (c->D == 1) ? Layout<1>::NF : (c->D == 2) ? Layout<2>::NF : NF3;
    if (c->D == 2) { // fastest measured on the double Mach reflection; pond_autotune re-picks
        c->bx = 8;
        c->by = 8;
    }
    const int64_t n = P.ncell, nf = P.nface;
    bool ok = true;
    auto alloc = [&](void **ptr, size_t bytes) {
        if (ok && hipMalloc(ptr, std::max<size_t>(bytes, 8)) != hipSuccess) ok = false;
    };
    alloc((void **)&c->U, sizeof(double) * (c->D + 2) * n);
    alloc(&c->H, c->rsize * c->nh * n);
    alloc(&c->F, c->rsize * c->nfp * nf);
    alloc((void **)&c->fiter, sizeof(int) * nf);
    alloc((void **)&c->cell_off, sizeof(int64_t) * (P.n_inst + 1));
    alloc((void **)&c->pad_off, sizeof(int64_t) * (P.n_inst + 1));
    alloc((void **)&c->t, sizeof(double) * P.n_inst);
    alloc((void **)&c->tstart, sizeof(double) * P.n_inst);
    alloc((void **)&c->dt, sizeof(double) * P.n_inst);
    P.vslots = (P.n_inst == 1) ? NSLOT : 1;
    alloc((void **)&c->vmax, sizeof(unsigned long long) * 2 * P.n_inst * P.vslots);
    alloc((void **)&c->stats, sizeof(unsigned long long) * ST_N * NSLOT);
    alloc((void **)&c->err, sizeof(int));
    alloc((void **)&c->inst_err, sizeof(int) * P.n_inst);
    // read-out staging, and the per-block records of the end-of-call summary
    alloc((void **)&c->scratch, sizeof(double) * std::max<int64_t>(4 * std::max(n, nf), (int64_t)SUM_BLOCKS * SUM3_NV));
    if (c->D == 3) alloc(&c->rec3, c->rsize * NR3 * n);
    if (cfg->flags & POND_FLAG_SEMI_LAGRANGIAN) {
        alloc((void **)&c->U2, sizeof(double) * (c->D + 2) * n);
        alloc(&c->H2, c->rsize * c->nh * n);
    }
    if (P.n_inst > 1) {
        alloc((void **)&c->cell_inst, sizeof(int) * n);
        alloc((void **)&c->face_inst, sizeof(int) * nf);
        alloc((void **)&c->dxk, sizeof(double) * P.n_inst);
    }
    if (c->D == 2) {
        int64_t cap = 0;
        for (const auto &t : kTiles2D) cap = std::max(cap, tail_cap_for(c, t.first, t.second));
        P.tail_cap = (int)cap;
        P.tail_n = 2 * NSLOT * cap;
        alloc((void **)&c->tail_f, sizeof(int) * P.tail_n);
        alloc((void **)&c->tail_meta, sizeof(int) * P.tail_n);
        alloc(&c->tail_s, c->rsize * 6 * P.tail_n);
        alloc((void **)&c->tail_count, sizeof(int) * 2 * NSLOT);
        alloc((void **)&c->tblock, sizeof(int) * n);
        // (measured on the 1920 x 480 double Mach reflection: finite volumes 4 in FP64 and 2
        // mixed; the semi-Lagrangian step 2 in both, 1.21 against 1.99 ms per step in FP64)
        P.iter_split = (cfg->flags & POND_FLAG_SEMI_LAGRANGIAN) ? 2 : (cfg->precision == POND_FP64) ? 4 : 2;
    }
    if (!ok) {
        free_all(c);
        delete c;
        return POND_ENOMEM;
    }
    if (hipStreamCreate(&c->own_stream) != hipSuccess) {
        free_all(c);
        delete c;
        return POND_EDEVICE;
    }
    c->stream = c->own_stream;
    // upload: primitive fields (staged through scratch), instance tables
    const int nprim = (c->D == 3) ? 5 : 4;
    std::vector<double> prim4((size_t)nprim * n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
        prim4[i] = rho[i];
        prim4[n + i] = ux[i];
        prim4[2 * n + i] = (c->D >= 2) ? uy[i] : 0.0;
        if (c->D == 3) prim4[3 * n + i] = uz[i];
        prim4[(nprim - 1) * n + i] = p[i];
    }
    std::vector<double> zeros(P.n_inst, 0.0);
    std::vector<unsigned long long> zv((size_t)2 * P.n_inst * P.vslots, 0ull), zs((size_t)ST_N * NSLOT, 0ull);
    bool up = hip_ok(hipMemcpy(c->scratch, prim4.data(), sizeof(double) * prim4.size(), hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->cell_off, coff.data(), sizeof(int64_t) * coff.size(), hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->pad_off, poff.data(), sizeof(int64_t) * poff.size(), hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->t, zeros.data(), sizeof(double) * P.n_inst, hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->tstart, zeros.data(), sizeof(double) * P.n_inst, hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->dt, zeros.data(), sizeof(double) * P.n_inst, hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->vmax, zv.data(), sizeof(unsigned long long) * zv.size(), hipMemcpyHostToDevice)) &&
              hip_ok(hipMemcpy(c->stats, zs.data(), sizeof(unsigned long long) * zs.size(), hipMemcpyHostToDevice)) &&
              hip_ok(hipMemset(c->err, 0, sizeof(int))) &&
              hip_ok(hipMemset(c->inst_err, 0, sizeof(int) * P.n_inst));
    if (up && P.n_inst > 1) {
        std::vector<int> ci(n), fi(nf);
        for (int k = 0; k < P.n_inst; ++k) {
            for (int64_t j = coff[k]; j < coff[k + 1]; ++j) ci[j] = k;
            for (int64_t f = coff[k] + k; f <= coff[k + 1] + k; ++f) fi[f] = k;
        }
        std::vector<double> dxv(P.n_inst);
        for (int k = 0; k < P.n_inst; ++k) dxv[k] = (cfg->x1 - cfg->x0) / len[k];
        up = hip_ok(hipMemcpy(c->cell_inst, ci.data(), sizeof(int) * n, hipMemcpyHostToDevice)) &&
             hip_ok(hipMemcpy(c->face_inst, fi.data(), sizeof(int) * nf, hipMemcpyHostToDevice)) &&
             hip_ok(hipMemcpy(c->dxk, dxv.data(), sizeof(double) * P.n_inst, hipMemcpyHostToDevice));
    }
    if (!up) {
        pond_free(c);
        return POND_EDEVICE;
    }
    c->tube_span = compute_span(c, c->bx);
    c->sl_span = compute_cell_span(c, 256);
    if (c->D == 1)
        c->precision == POND_FP64 ? init_launch<1, double>(c, c->scratch) : init_launch<1, float>(c, c->scratch);
    else if (c->D == 2)
        c->precision == POND_FP64 ? init_launch<2, double>(c, c->scratch) : init_launch<2, float>(c, c->scratch);
    else if (c->precision == POND_FP64)
        init_kernel_3d<double><<<blocks(std::max(n, nf), 256), 256, 0, c->stream>>>(c->P, c->G3, state_of<double>(c), c->scratch);
    else
        init_kernel_3d<float><<<blocks(std::max(n, nf), 256), 256, 0, c->stream>>>(c->P, c->G3, state_of<float>(c), c->scratch);
    if (!hip_ok(hipGetLastError()) || !hip_ok(hipStreamSynchronize(c->stream))) {
        pond_free(c);
        return POND_EDEVICE;
    }
    *out = c;
    return POND_OK;
}

pond_status pond_step(pond_ctx *c, int32_t nsteps, double t_end, pond_stats *st)
{
    if (!c || nsteps < 0) return POND_EINVAL;
    if (c->cfg.seed_mode == POND_SEED_MLP && !c->mlp.ready) return POND_ESTATE;
    // counters and error flags describe this call only (frozen instances stay frozen
    // through inst_err, and their cells are not updated again, so they raise no new flag)
    HIPCHK(hipMemsetAsync(c->stats, 0, sizeof(unsigned long long) * ST_N * NSLOT, c->stream));
    HIPCHK(hipMemsetAsync(c->err, 0, sizeof(int), c->stream));
    double kt[5] = {0, 0, 0, 0, 0};
    if (c->timing) {
        size_t need = (size_t)6 * std::max(nsteps, 1);
        while (c->evs.size() < need) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->evs.push_back(e);
        }
    }
    int s0 = 0;
    if (c->resident && !c->timing && nsteps > 0 && c->cfg.seed_mode != POND_SEED_MLP && !semi_lagrangian(c)) {
        HIPCHK(c->precision == POND_FP64 ? launch_resident<double>(c, nsteps, t_end)
                                         : launch_resident<float>(c, nsteps, t_end));
        s0 = nsteps;
    } else if (c->use_graph && !c->timing && nsteps >= 2) {
        if (!c->gexec || c->g_tend != t_end || c->g_slot != c->slot) {
            drop_graph(c);
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e1 = step_once(c, t_end);
            hipError_t e2 = step_once(c, t_end); // two steps: the step parity returns
            hipError_t e3 = hipStreamEndCapture(c->stream, &g);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return POND_EDEVICE;
            }
            hipError_t e4 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e4 != hipSuccess) {
                c->gexec = nullptr;
                return POND_EDEVICE;
            }
            c->g_tend = t_end;
            c->g_slot = c->slot;
        }
        for (; s0 + 2 <= nsteps; s0 += 2) HIPCHK(hipGraphLaunch(c->gexec, c->stream));
    }
    for (int s = s0; s < nsteps; ++s) {
        c->ev = c->timing ? &c->evs[(size_t)6 * s] : nullptr;
        HIPCHK(step_once(c, t_end));
    }
    if (c->timing && nsteps > 0) {
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int s = 0; s < nsteps; ++s) {
            hipEvent_t *e = &c->evs[(size_t)6 * s];
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e[0], e[1]);
            kt[0] += ms;
            (void)hipEventElapsedTime(&ms, e[2], e[3]);
            kt[1] += ms;
            (void)hipEventElapsedTime(&ms, e[4], e[5]);
            kt[2] += ms;
            (void)hipEventElapsedTime(&ms, e[1], e[2]);
            kt[3] += ms;
            (void)hipEventElapsedTime(&ms, e[3], e[4]);
            kt[4] += ms;
        }
        for (int q = 0; q < 5; ++q) c->ktime[q] = kt[q] / nsteps;
    }
    c->ev = nullptr;
    std::vector<unsigned long long> hsl((size_t)ST_N * NSLOT);
    int herr = 0;
    HIPCHK(hipMemcpyAsync(hsl.data(), c->stats, sizeof(unsigned long long) * hsl.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&herr, c->err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    std::vector<double> ht(c->P.n_inst), hdt(c->P.n_inst);
    HIPCHK(hipMemcpyAsync(ht.data(), c->t, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(hdt.data(), c->dt, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToHost, c->stream));
    std::vector<int> fe(c->P.n_inst);
    HIPCHK(hipMemcpyAsync(fe.data(), c->inst_err, sizeof(int) * c->P.n_inst, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> sum;
    if (st) {
        // summary of the state after the call: one record per block of summary_kernel
        const int nv = (c->D == 3) ? SUM3_NV : SUM_NV;
        sum.resize((size_t)SUM_BLOCKS * nv);
        if (c->D == 1)
            summary_kernel<1><<<SUM_BLOCKS, 256, 0, c->stream>>>(c->P, c->U, c->fiter, c->dxk, c->cell_inst, c->scratch);
        else if (c->D == 2)
            summary_kernel<2><<<SUM_BLOCKS, 256, 0, c->stream>>>(c->P, c->U, c->fiter, c->dxk, c->cell_inst, c->scratch);
        else
            summary_kernel_3d<<<SUM_BLOCKS, 256, 0, c->stream>>>(c->P, c->G3, c->U, c->fiter, c->scratch);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(sum.data(), c->scratch, sizeof(double) * sum.size(), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    c->steps_done += nsteps;
    unsigned long long hs[ST_N];
    for (int q = 0; q < ST_N; ++q) {
        unsigned long long a = 0;
        for (int w = 0; w < NSLOT; ++w) {
            const unsigned long long v = hsl[(size_t)q * NSLOT + w];
            a = (q == ST_ITMAX) ? std::max(a, v) : a + v;
        }
        hs[q] = a;
    }
    if (st) {
        memset(st, 0, sizeof(*st));
        st->steps = nsteps;
        st->cell_updates = (int64_t)hs[ST_CELLS];
        st->converged_cell_updates = (int64_t)hs[ST_CONV_CELLS];
        st->faces = (int64_t)hs[ST_FACES];
        st->iters_total = (int64_t)hs[ST_ITERS];
        st->iters_max = (int32_t)hs[ST_ITMAX];
        st->nonconverged = (int64_t)hs[ST_NONCONV];
        st->fallback = (int64_t)hs[ST_FALLBACK];
        st->departure_out = (int64_t)hs[ST_DEPOUT];
        st->tail_faces = (int64_t)hs[ST_TAIL_FACES];
        st->tail_iters = (int64_t)hs[ST_TAIL_ITERS];
        st->t_min = *std::min_element(ht.begin(), ht.end());
        st->t_max = *std::max_element(ht.begin(), ht.end());
        st->dt_min = *std::min_element(hdt.begin(), hdt.end());
        st->dt_max = *std::max_element(hdt.begin(), hdt.end());
        st->failed_instances = (int32_t)std::count_if(fe.begin(), fe.end(), [](int v) { return v != 0; });
        st->first_failed_instance = -1;
        for (int k = 0; k < c->P.n_inst; ++k)
            if (fe[k] && !(k < (int)c->h_failed.size() && c->h_failed[k])) {
                st->first_failed_instance = k;
                break;
            }
        // records: rho_min, T_min, the conserved totals (4, or 5 in 3D), bad cell, face
        const int nv = (c->D == 3) ? SUM3_NV : SUM_NV, nt = nv - 4;
        double rmin = INFINITY, tmin = INFINITY, bad = INFINITY, nonc = INFINITY, tot[5] = {0, 0, 0, 0, 0};
        for (int b = 0; b < SUM_BLOCKS; ++b) {
            const double *r = &sum[(size_t)b * nv];
            rmin = std::fmin(rmin, r[0]);
            tmin = std::fmin(tmin, r[1]);
            for (int q = 0; q < nt; ++q) tot[q] += r[2 + q];
            bad = std::fmin(bad, r[2 + nt]);
            nonc = std::fmin(nonc, r[3 + nt]);
        }
        st->rho_min = rmin;
        st->T_min = tmin;
        for (int q = 0; q < 5; ++q) st->totals[q] = tot[q];
        st->first_failed_cell = std::isfinite(bad) ? (int64_t)bad : -1;
        st->first_nonconv_face = std::isfinite(nonc) ? (int64_t)nonc : -1;
    }
    c->h_failed = fe;
    if (herr & ERR_NONPHYS) return POND_ENONPHYS;
    if ((c->cfg.flags & POND_FLAG_STRICT) && hs[ST_NONCONV]) return POND_ENOCONV;
    if ((c->cfg.flags & POND_FLAG_STRICT) && (herr & ERR_DEPART)) return POND_ECFL;
    return POND_OK;
}

pond_status pond_moments_device(const pond_ctx *c, double *dev_out)
{
    if (!c || !dev_out) return POND_EINVAL;
    int64_t n = c->P.ncell;
    if (c->D == 1)
        fields_kernel<1><<<blocks(n, 256), 256, 0, c->stream>>>(n, c->U, c->P.Cv, dev_out);
    else if (c->D == 2)
        fields_kernel<2><<<blocks(n, 256), 256, 0, c->stream>>>(n, c->U, c->P.Cv, dev_out);
    else
        fields_kernel_3d<<<blocks(n, 256), 256, 0, c->stream>>>(n, c->U, c->P.Cv, dev_out);
    HIPCHK(hipGetLastError());
    return POND_OK;
}

pond_status pond_moments(const pond_ctx *c, double *rho, double *ux, double *uy, double *T)
{
    if (!c || !rho || !ux || !T) return POND_EINVAL;
    pond_status s = pond_moments_device(c, c->scratch);
    if (s != POND_OK) return s;
    int64_t n = c->P.ncell;
    std::vector<double> h((size_t)4 * n);
    HIPCHK(hipMemcpyAsync(h.data(), c->scratch, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    memcpy(rho, h.data(), sizeof(double) * n);
    memcpy(ux, h.data() + n, sizeof(double) * n);
    if (uy) memcpy(uy, h.data() + 2 * n, sizeof(double) * n);
    memcpy(T, h.data() + 3 * n, sizeof(double) * n);
    return POND_OK;
}

// ---- checkpoint: the carried state of a context, in a flat binary file ----

namespace {

struct CkptHeader {
    char magic[8];
    int32_t abi, dim, precision, n_inst, nh, nfp, vslots, slot, iter_split, pad;
    int64_t ncell, nface, steps_done;
};

struct Blob {
    void *dev;
    size_t bytes;
};

std::vector<Blob> ckpt_blobs(pond_ctx *c)
{
    const int64_t n = c->P.ncell, nf = c->P.nface, ni = c->P.n_inst;
    return {{c->U, sizeof(double) * (c->D + 2) * n},
            {c->H, c->rsize * c->nh * n},
            {c->F, c->rsize * c->nfp * nf},
            {c->fiter, sizeof(int) * nf},
            {c->t, sizeof(double) * ni},
            {c->tstart, sizeof(double) * ni},
            {c->dt, sizeof(double) * ni},
            {c->vmax, sizeof(unsigned long long) * 2 * ni * c->P.vslots},
            {c->inst_err, sizeof(int) * ni}};
}

CkptHeader ckpt_header(const pond_ctx *c)
{
    CkptHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, "PONDCKP1", 8);
    h.abi = POND_ABI_VERSION;
    h.dim = c->D;
    h.precision = c->precision;
    h.n_inst = c->P.n_inst;
    h.nh = c->nh;
    h.nfp = c->nfp;
    h.vslots = c->P.vslots;
    h.slot = c->slot;
    h.iter_split = c->P.iter_split;
    h.ncell = c->P.ncell;
    h.nface = c->P.nface;
    h.steps_done = c->steps_done;
    return h;
}

} // namespace

pond_status pond_save(pond_ctx *c, const char *path)
{
    if (!c || !path || c->layout != POND_LAYOUT_HERMITE) return POND_EINVAL;
    FILE *fp = fopen(path, "wb");
    if (!fp) return POND_EINVAL;
    CkptHeader h = ckpt_header(c);
    bool ok = fwrite(&h, sizeof(h), 1, fp) == 1;
    std::vector<unsigned char> buf;
    for (const Blob &b : ckpt_blobs(c)) {
        if (!ok) break;
        buf.resize(b.bytes);
        if (hipMemcpyAsync(buf.data(), b.dev, b.bytes, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess) {
            fclose(fp);
            return POND_EDEVICE;
        }
        ok = fwrite(buf.data(), 1, b.bytes, fp) == b.bytes;
    }
    ok = (fclose(fp) == 0) && ok;
    return ok ? POND_OK : POND_EINVAL;
}

pond_status pond_load(pond_ctx *c, const char *path)
{
    if (!c || !path || c->layout != POND_LAYOUT_HERMITE) return POND_EINVAL;
    FILE *fp = fopen(path, "rb");
    if (!fp) return POND_EINVAL;
    CkptHeader h, mine = ckpt_header(c);
    bool ok = fread(&h, sizeof(h), 1, fp) == 1 && memcmp(h.magic, mine.magic, 8) == 0 &&
              h.abi == mine.abi && h.dim == mine.dim &&
              (h.precision == POND_FP64 || h.precision == POND_MIXED) &&
              h.n_inst == mine.n_inst && h.nh == mine.nh && h.nfp == mine.nfp &&
              h.vslots == mine.vslots && h.ncell == mine.ncell && h.nface == mine.nface;
    // a checkpoint of the other precision: its coefficient and face planes (blobs 1 and 2)
    // hold the other element size and are converted on the way in
    const bool convert = ok && h.precision != mine.precision;
    const size_t fsize = (h.precision == POND_FP64) ? sizeof(double) : sizeof(float);
    std::vector<std::vector<unsigned char>> data;
    int kb = 0;
    for (const Blob &b : ckpt_blobs(c)) {
        if (!ok) break;
        const bool planes = convert && (kb == 1 || kb == 2);
        const size_t count = b.bytes / c->rsize;
        std::vector<unsigned char> raw(planes ? count * fsize : b.bytes);
        ok = fread(raw.data(), 1, raw.size(), fp) == raw.size();
        if (ok && planes) {
            std::vector<unsigned char> conv(b.bytes);
            for (size_t q = 0; q < count; ++q) {
                if (fsize == sizeof(double)) {
                    double v;
                    memcpy(&v, raw.data() + q * sizeof(double), sizeof(double));
                    float w = (float)v;
                    memcpy(conv.data() + q * sizeof(float), &w, sizeof(float));
                } else {
                    float v;
                    memcpy(&v, raw.data() + q * sizeof(float), sizeof(float));
                    double w = (double)v;
                    memcpy(conv.data() + q * sizeof(double), &w, sizeof(double));
                }
            }
            raw.swap(conv);
        }
        data.push_back(std::move(raw));
        ++kb;
    }
    fclose(fp);
    if (!ok) return POND_EINVAL; // the context is left as it was
    drop_graph(c);
    const std::vector<Blob> blobs = ckpt_blobs(c);
    for (size_t k = 0; k < blobs.size(); ++k)
        HIPCHK(hipMemcpyAsync(blobs[k].dev, data[k].data(), blobs[k].bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->h_failed.assign(c->P.n_inst, 0);
    HIPCHK(hipMemcpy(c->h_failed.data(), c->inst_err, sizeof(int) * c->P.n_inst, hipMemcpyDeviceToHost));
    c->slot = h.slot;
    if (!convert) c->P.iter_split = h.iter_split; // the other precision's hand-over point is not taken
    c->steps_done = h.steps_done;
    return POND_OK;
}

pond_status pond_conserved(const pond_ctx *c, double *U)
{
    if (!c || !U) return POND_EINVAL;
    HIPCHK(hipMemcpyAsync(U, c->U, sizeof(double) * (c->D + 2) * c->P.ncell, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return POND_OK;
}

pond_status pond_populations(const pond_ctx *c, double *f, double *g, double *frame)
{
    if (!c || !f || !g || !frame || c->layout != POND_LAYOUT_HERMITE) return POND_EINVAL;
    const int64_t n = c->P.ncell;
    const int Q = (c->D == 1) ? 4 : (c->D == 2) ? 16 : 64;
    double *df = nullptr, *dg = nullptr, *dfr = nullptr;
    size_t nb = sizeof(double) * (size_t)n;
    if (hipMalloc(&df, nb * Q) != hipSuccess || hipMalloc(&dg, nb * Q) != hipSuccess ||
        hipMalloc(&dfr, nb * (c->D + 1)) != hipSuccess) {
        if (df) (void)hipFree(df);
        if (dg) (void)hipFree(dg);
        return POND_ENOMEM;
    }
    pond_ctx *m = const_cast<pond_ctx *>(c);
    if (c->D == 3) {
        if (c->precision == POND_FP64)
            pops_kernel_3d<double><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), df, dg, dfr);
        else
            pops_kernel_3d<float><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), df, dg, dfr);
    } else if (c->D == 1) {
        if (c->precision == POND_FP64)
            pops_kernel<1, double><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), df, dg, dfr);
        else
            pops_kernel<1, float><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), df, dg, dfr);
    } else {
        const bool r1 = reg_of(c) != 0;
        if (c->precision == POND_FP64 && r1)
            pops_kernel<2, double, 1><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), df, dg, dfr);
        else if (c->precision == POND_FP64)
            pops_kernel<2, double, 0><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), df, dg, dfr);
        else if (r1)
            pops_kernel<2, float, 1><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), df, dg, dfr);
        else
            pops_kernel<2, float, 0><<<blocks(n, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), df, dg, dfr);
    }
    bool ok = hip_ok(hipGetLastError()) &&
              hip_ok(hipMemcpyAsync(f, df, nb * Q, hipMemcpyDeviceToHost, c->stream)) &&
              hip_ok(hipMemcpyAsync(g, dg, nb * Q, hipMemcpyDeviceToHost, c->stream)) &&
              hip_ok(hipMemcpyAsync(frame, dfr, nb * (c->D + 1), hipMemcpyDeviceToHost, c->stream)) &&
              hip_ok(hipStreamSynchronize(c->stream));
    (void)hipFree(df);
    (void)hipFree(dg);
    (void)hipFree(dfr);
    return ok ? POND_OK : POND_EDEVICE;
}

int64_t pond_nfaces(const pond_ctx *c) { return c ? c->P.nface : 0; }

pond_status pond_face_frames(const pond_ctx *c, double *out)
{
    if (!c || !out) return POND_EINVAL;
    const int64_t nf = c->P.nface;
    const int nv = c->D + 1;
    std::vector<unsigned char> buf(c->rsize * nv * nf);
    HIPCHK(hipMemcpyAsync(buf.data(), c->F, buf.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int v = 0; v < nv; ++v)
        for (int64_t f = 0; f < nf; ++f)
            out[f * nv + v] = (c->precision == POND_FP64)
                                  ? reinterpret_cast<const double *>(buf.data())[v * nf + f]
                                  : (double)reinterpret_cast<const float *>(buf.data())[v * nf + f];
    return POND_OK;
}

pond_status pond_set_face_frames(pond_ctx *c, const double *in)
{
    if (!c || !in) return POND_EINVAL;
    const int64_t nf = c->P.nface;
    const int nv = c->D + 1;
    std::vector<unsigned char> buf(c->rsize * nv * nf);
    for (int v = 0; v < nv; ++v)
        for (int64_t f = 0; f < nf; ++f) {
            double x = in[f * nv + v];
            if (v == nv - 1 && !(x > 0.0)) x = -1.0;
            if (c->precision == POND_FP64)
                reinterpret_cast<double *>(buf.data())[v * nf + f] = x;
            else
                reinterpret_cast<float *>(buf.data())[v * nf + f] = (float)x;
        }
    HIPCHK(hipMemcpyAsync(c->F, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return POND_OK;
}

pond_status pond_face_moments(const pond_ctx *c, double *Mf, double *Mg)
{
    if (!c || !Mf || !Mg) return POND_EINVAL;
    const int64_t nf = c->P.nface;
    const int nf3 = (c->D == 1) ? 4 : (c->D == 2) ? 15 : 40, ng2 = (c->D == 1) ? 3 : (c->D == 2) ? 7 : 13;
    double *dm = nullptr, *dg = nullptr;
    if (hipMalloc(&dm, sizeof(double) * nf3 * nf) != hipSuccess ||
        hipMalloc(&dg, sizeof(double) * ng2 * nf) != hipSuccess) {
        if (dm) (void)hipFree(dm);
        return POND_ENOMEM;
    }
    pond_ctx *m = const_cast<pond_ctx *>(c);
    if (c->D == 3) {
        if (c->precision == POND_FP64)
            face_moments_kernel_3d<double><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), dm, dg);
        else
            face_moments_kernel_3d<float><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), dm, dg);
    } else if (c->D == 1) {
        if (c->precision == POND_FP64)
            face_moments_kernel<1, double><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), dm, dg);
        else
            face_moments_kernel<1, float><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), dm, dg);
    } else {
        if (c->precision == POND_FP64)
            face_moments_kernel<2, double><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<double>(m), dm, dg);
        else
            face_moments_kernel<2, float><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<float>(m), dm, dg);
    }
    bool ok = hip_ok(hipGetLastError()) &&
              hip_ok(hipMemcpyAsync(Mf, dm, sizeof(double) * nf3 * nf, hipMemcpyDeviceToHost, c->stream)) &&
              hip_ok(hipMemcpyAsync(Mg, dg, sizeof(double) * ng2 * nf, hipMemcpyDeviceToHost, c->stream)) &&
              hip_ok(hipStreamSynchronize(c->stream));
    (void)hipFree(dm);
    (void)hipFree(dg);
    return ok ? POND_OK : POND_EDEVICE;
}

pond_status pond_face_iters(const pond_ctx *c, int32_t *out)
{
    if (!c || !out) return POND_EINVAL;
    const int64_t nf = c->P.nface;
    std::vector<int> h(nf);
    HIPCHK(hipMemcpyAsync(h.data(), c->fiter, sizeof(int) * nf, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int64_t f = 0; f < nf; ++f) {
        int it = h[f] & 0xffff;
        out[f] = ((h[f] >> 16) & 1) ? -it : it;
    }
    return POND_OK;
}

pond_status pond_failed_instances(const pond_ctx *c, int32_t *flags)
{
    if (!c || !flags) return POND_EINVAL;
    HIPCHK(hipMemcpyAsync(flags, c->inst_err, sizeof(int) * c->P.n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return POND_OK;
}

pond_status pond_time(const pond_ctx *c, double *t)
{
    if (!c || !t) return POND_EINVAL;
    HIPCHK(hipMemcpyAsync(t, c->t, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return POND_OK;
}

pond_status pond_set_stream(pond_ctx *c, void *s)
{
    if (!c) return POND_EINVAL;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->stream = s ? (hipStream_t)s : c->own_stream;
    return POND_OK;
}

pond_status pond_set_tiles(pond_ctx *c, int32_t bx, int32_t by, int32_t cell_block)
{
    if (!c || c->D == 3) return POND_EINVAL;
    // every kernel is compiled for blocks of at most 256 threads
    if (cell_block < 64 || cell_block > 256 || cell_block % 64) return POND_EINVAL;
    if (c->D == 1) {
        if (bx < 64 || bx > 256 || bx % 64 || by != 1) return POND_EINVAL;
    } else {
        if (bx < 1 || by < 1 || bx * by > 256 || (bx * by) % 64) return POND_EINVAL;
    }
    int span = compute_span(c, bx);
    if (face_lds_bytes(c, bx, by, span) > 160 * 1024) return POND_EINVAL;
    if (c->D == 2 && !ensure_tail(c, bx, by)) return POND_ENOMEM;
    drop_graph(c);
    c->bx = bx;
    c->by = by;
    c->cell_block = cell_block;
    c->tube_span = span;
    return POND_OK;
}

pond_status pond_set_graph(pond_ctx *c, int32_t on)
{
    if (!c) return POND_EINVAL;
    c->use_graph = on ? 1 : 0;
    if (!on) drop_graph(c);
    return POND_OK;
}

pond_status pond_set_resident(pond_ctx *c, int32_t on)
{
    if (!c || (on && (c->D != 1 || semi_lagrangian(c)))) return POND_EINVAL;
    if (on && !c->res_order) {
        // longest tubes first, so that the last blocks to start are the short ones
        const int n = c->P.n_inst;
        std::vector<int> ord(n);
        for (int k = 0; k < n; ++k) ord[k] = k;
        const auto &off = c->h_cell_off;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
        int *d = nullptr;
        if (hipMalloc(&d, sizeof(int) * n) != hipSuccess) return POND_ENOMEM;
        if (!hip_ok(hipMemcpy(d, ord.data(), sizeof(int) * n, hipMemcpyHostToDevice))) {
            (void)hipFree(d);
            return POND_EDEVICE;
        }
        c->res_order = d;
    }
    c->resident = on ? 1 : 0;
    return POND_OK;
}

pond_status pond_set_iter_split(pond_ctx *c, int32_t k)
{
    if (!c || k < 0 || c->D == 3) return POND_EINVAL;
    drop_graph(c);
    if (c->D == 2) c->P.iter_split = k;
    return POND_OK;
}

pond_status pond_set_state_layout(pond_ctx *c, int32_t layout)
{
    if (!c || (layout != POND_LAYOUT_HERMITE && layout != POND_LAYOUT_POPULATIONS)) return POND_EINVAL;
    if (layout == c->layout) return POND_OK;
    if (c->D != 2 || semi_lagrangian(c) || reg_of(c) || c->P.limiter != POND_LIM_VANLEER ||
        c->cfg.seed_mode != POND_SEED_PREV)
        return POND_EINVAL;
    drop_graph(c);
    const int64_t n = c->P.ncell;
    const int nh = layout == POND_LAYOUT_POPULATIONS ? NPOP2 : Layout<2>::NH;
    void *dst = nullptr;
    if (hipMalloc(&dst, c->rsize * nh * n) != hipSuccess) return POND_ENOMEM;
    const bool to_pops = layout == POND_LAYOUT_POPULATIONS;
    if (c->precision == POND_FP64) {
        if (to_pops)
            coef_to_pops_kernel_2d<double><<<blocks(n, 256), 256, 0, c->stream>>>(
                c->P, c->U, static_cast<const double *>(c->H), static_cast<double *>(dst));
        else
            pops_to_coef_kernel_2d<double><<<blocks(n, 256), 256, 0, c->stream>>>(
                c->P, static_cast<const double *>(c->H), static_cast<double *>(dst));
    } else {
        if (to_pops)
            coef_to_pops_kernel_2d<float><<<blocks(n, 256), 256, 0, c->stream>>>(
                c->P, c->U, static_cast<const float *>(c->H), static_cast<float *>(dst));
        else
            pops_to_coef_kernel_2d<float><<<blocks(n, 256), 256, 0, c->stream>>>(
                c->P, static_cast<const float *>(c->H), static_cast<float *>(dst));
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipFree(dst);
        return POND_EDEVICE;
    }
    (void)hipFree(c->H);
    c->H = dst;
    c->nh = nh;
    c->layout = layout;
    return POND_OK;
}

pond_status pond_get_tiles(const pond_ctx *c, int32_t *bx, int32_t *by, int32_t *cell_block)
{
    if (!c || !bx || !by || !cell_block) return POND_EINVAL;
    *bx = c->bx;
    *by = c->by;
    *cell_block = c->cell_block;
    return POND_OK;
}

pond_status pond_autotune(pond_ctx *c)
{
    if (!c) return POND_EINVAL;
    if (c->D == 3 || semi_lagrangian(c)) return POND_OK; // one launch shape in 3D and for the SL kernels
    // the face kernel is the dominant cost; time it on the current state. It only writes
    // face state, which is saved first and restored afterwards (the next step's seeds).
    const size_t fbytes = c->rsize * c->nfp * c->P.nface;
    void *save = nullptr;
    const size_t ibytes = sizeof(int) * c->P.nface;
    HIPCHK(hipMalloc(&save, fbytes + ibytes + sizeof(int)));
    int *save_iter = reinterpret_cast<int *>(static_cast<char *>(save) + fbytes);
    HIPCHK(hipMemcpyAsync(save, c->F, fbytes, hipMemcpyDeviceToDevice, c->stream));
    // the iteration counts (read by the learned seed's face selection) and the error flags
    // are restored as well
    HIPCHK(hipMemcpyAsync(save_iter, c->fiter, ibytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(save_iter + c->P.nface, c->err, sizeof(int), hipMemcpyDeviceToDevice, c->stream));
    // a dt must exist for the face kernel: run the dt kernel's effect on a copy
    std::vector<std::pair<int, int>> cand;
    if (c->D == 1)
        cand = {{64, 1}, {128, 1}, {256, 1}};
    else
        cand.assign(std::begin(kTiles2D), std::end(kTiles2D));
    double best = 1e30;
    int bbx = c->bx, bby = c->by;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    // make sure dt > 0: use the time step the next step would take
    double *sdt = nullptr;
    (void)hipMalloc(&sdt, sizeof(double) * c->P.n_inst * 3);
    (void)hipMemcpyAsync(sdt, c->dt, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(sdt + c->P.n_inst, c->t, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(sdt + 2 * c->P.n_inst, c->tstart, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToDevice, c->stream);
    {
        State<double> S = state_of<double>(c);
        // the dt kernel only touches t, tstart, dt and the other vmax slot: all restored below
        std::vector<unsigned long long> vm((size_t)2 * c->P.n_inst * c->P.vslots);
        (void)hipMemcpyAsync(vm.data(), c->vmax, sizeof(unsigned long long) * vm.size(), hipMemcpyDeviceToHost, c->stream);
        (void)hipStreamSynchronize(c->stream);
        dt_kernel<1, double><<<c->P.n_inst, 64, 0, c->stream>>>(c->P, S, INFINITY, c->slot);
        for (auto &cd : cand) {
            if (c->D == 2 && ((cd.first * cd.second) % 64 != 0)) continue;
            if (face_lds_bytes(c, cd.first, cd.second, compute_span(c, cd.first)) > 160 * 1024) continue;
            // the fastest of 4 timed launches after a warm-up one: shapes whose times differ
            // by a per cent or two are told apart more reliably by the minimum than by a sum
            double tmin = 1e30;
            for (int rep = 0; rep < 5; ++rep) {
                (void)hipMemcpyAsync(c->F, save, fbytes, hipMemcpyDeviceToDevice, c->stream);
                hipEventRecord(e0, c->stream);
                if (face_once(c, cd.first, cd.second) != hipSuccess) {
                    tmin = 1e30;
                    break;
                }
                hipEventRecord(e1, c->stream);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) tmin = std::min(tmin, (double)ms);
            }
            if (tmin < best) {
                best = tmin;
                bbx = cd.first;
                bby = cd.second;
            }
        }
        (void)hipMemcpyAsync(c->vmax, vm.data(), sizeof(unsigned long long) * vm.size(), hipMemcpyHostToDevice, c->stream);
    }
    (void)hipMemcpyAsync(c->dt, sdt, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->t, sdt + c->P.n_inst, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->tstart, sdt + 2 * c->P.n_inst, sizeof(double) * c->P.n_inst, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->F, save, fbytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->fiter, save_iter, ibytes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(c->err, save_iter + c->P.nface, sizeof(int), hipMemcpyDeviceToDevice, c->stream);
    HIPCHK(hipMemsetAsync(c->stats, 0, sizeof(unsigned long long) * ST_N * NSLOT, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    (void)hipFree(sdt);
    (void)hipFree(save);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return pond_set_tiles(c, bbx, bby, c->cell_block);
}

pond_status pond_enable_timing(pond_ctx *c, int32_t on)
{
    if (!c) return POND_EINVAL;
    c->timing = on ? 1 : 0;
    return POND_OK;
}

pond_status pond_kernel_times(const pond_ctx *c, double *out)
{
    if (!c || !out) return POND_EINVAL;
    for (int q = 0; q < 5; ++q) out[q] = c->ktime[q];
    return POND_OK;
}

void pond_free(pond_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    free_all(c);
    for (auto &e : c->evs) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

} // extern "C"

// ---------------------------------------------------------------------------------------
// learned seed
// ---------------------------------------------------------------------------------------

struct pond_mlp {
    MlpDevice dev;
    hipStream_t stream = nullptr;
    int device = 0; // the device current at pond_mlp_create, which holds the buffers
};

namespace {

uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double unit_open(uint64_t &x) { return ((splitmix64(x) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

void he_init(std::vector<float> &p, uint64_t seed)
{
    std::fill(p.begin(), p.end(), 0.0f);
    uint64_t st = seed;
    auto fill = [&](int off, int rows, int cols) {
        double sd = std::sqrt(2.0 / cols);
        for (int i = 0; i < rows * cols; ++i) {
            double u1 = unit_open(st), u2 = unit_open(st);
            p[off + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    };
    fill(OFF_W1, MLP_H, MLP_NF);  // only the used inputs get weights; padding columns stay 0
    for (int o = MLP_H - 1; o >= 0; --o)
        for (int k = MLP_IN - 1; k >= 0; --k) p[OFF_W1 + o * MLP_IN + k] = (k < MLP_NF) ? p[OFF_W1 + o * MLP_NF + k] : 0.0f;
    fill(OFF_W2, MLP_H, MLP_H);
    fill(OFF_W3, MLP_OUT, MLP_H);
}

pond_status mlp_alloc(MlpDevice &M, int npartial)
{
    bool ok = hipMalloc(&M.master, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&M.adam_m, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&M.adam_v, sizeof(float) * MLP_NPARAM) == hipSuccess &&
              hipMalloc(&M.wbf, sizeof(__bf16) * (2 * MLP_H * MLP_IN + 16 * MLP_H)) == hipSuccess &&
              hipMalloc(&M.partial, sizeof(float) * (size_t)npartial * (MLP_NPARAM + 1)) == hipSuccess &&
              hipMalloc(&M.grad, sizeof(float) * (MLP_NPARAM + 1)) == hipSuccess;
    M.npartial = npartial;
    if (!ok) {
        mlp_free(M);
        return POND_ENOMEM;
    }
    return POND_OK;
}

pond_status mlp_upload(MlpDevice &M, const float *params, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(M.master, params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(M.adam_m, 0, sizeof(float) * MLP_NPARAM, st));
    HIPCHK(hipMemsetAsync(M.adam_v, 0, sizeof(float) * MLP_NPARAM, st));
    mlp_pack_kernel<<<blocks(MLP_H * MLP_IN, 256), 256, 0, st>>>(M.master, M.wbf);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    M.adam_t = 0;
    M.ready = true;
    return POND_OK;
}

int train_grid(int64_t n, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 31) / 32, cap)); }

// One epoch of Adam steps over consecutive batches of B samples; the loss of batch b is
// copied to dloss[b] (device). Returns the number of batches.
int train_epoch(MlpDevice &M, const float *X, const float *T, int64_t n, const pond_train_cfg *cfg,
                hipStream_t st, float *dloss)
{
    const int64_t B = cfg->batch;
    int nb = 0;
    for (int64_t b0 = 0; b0 < n; b0 += B) {
        int64_t nbn = std::min<int64_t>(B, n - b0);
        int nw = train_grid(nbn, M.npartial);
        mlp_train_kernel<<<nw, 64, 0, st>>>(M.wbf, M.master, X + b0 * MLP_IN, T + b0 * 4, nbn, M.partial);
        mlp_reduce_kernel<<<blocks(MLP_NPARAM + 1, 256), 256, 0, st>>>(M.partial, nw, M.grad);
        M.adam_t += 1;
        mlp_adam_kernel<<<blocks(MLP_NPARAM, 256), 256, 0, st>>>(M.master, M.adam_m, M.adam_v, M.grad, M.wbf,
                                                                 cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, M.adam_t);
        (void)hipMemcpyAsync(dloss + nb, M.grad + MLP_NPARAM, sizeof(float), hipMemcpyDeviceToDevice, st);
        ++nb;
    }
    return nb;
}

bool train_args_ok(const pond_mlp *m, const float *X, const float *T, int64_t n, const pond_train_cfg *cfg)
{
    return m && X && T && cfg && n >= 1 && cfg->epochs >= 0 && cfg->batch >= 32 && cfg->batch % 32 == 0;
}

} // namespace

// Batch losses and epoch means of pond_mlp_train_noalloc: a file-scope device array, one
// copy per device the library runs on (each holds it until the process ends). Host code
// reaches it only through the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float scratch[POND_NOALLOC_MAX_BATCHES + POND_NOALLOC_MAX_EPOCHS];

namespace {

constexpr int kMaxDevices = 64;
float *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// the device address of `scratch` on device `dev` (which must be current), looked up once
float *noalloc_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch[dev] = static_cast<float *>(ptr);
    }
    return g_scratch[dev];
}

// mean of the nb batch losses, summed in double in batch order (the arithmetic of
// pond_mlp_train's host loop), into out[0]
__global__ void loss_mean_kernel(const float *dloss, int nb, float *out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double sum = 0.0;
    for (int b = 0; b < nb; ++b) sum += (double)dloss[b];
    out[0] = (float)(sum / (nb > 1 ? nb : 1));
}

} // namespace

extern "C" {

int32_t pond_mlp_nparams(void) { return MLP_NPARAM; }

pond_status pond_mlp_create(const float *params, uint64_t seed, pond_mlp **out)
{
    if (!out) return POND_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return POND_EDEVICE;
    pond_mlp *m = new (std::nothrow) pond_mlp();
    if (!m) return POND_ENOMEM;
    if (hipGetDevice(&m->device) != hipSuccess || hipStreamCreate(&m->stream) != hipSuccess) {
        delete m;
        return POND_EDEVICE;
    }
    pond_status s = mlp_alloc(m->dev, 1024);
    if (s != POND_OK) {
        pond_mlp_free(m);
        return s;
    }
    std::vector<float> p(MLP_NPARAM);
    if (params)
        std::copy(params, params + MLP_NPARAM, p.begin());
    else
        he_init(p, seed);
    s = mlp_upload(m->dev, p.data(), m->stream);
    if (s != POND_OK) {
        pond_mlp_free(m);
        return s;
    }
    *out = m;
    return POND_OK;
}

pond_status pond_mlp_get(const pond_mlp *m, float *params)
{
    if (!m || !params) return POND_EINVAL;
    HIPCHK(hipMemcpyAsync(params, m->dev.master, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return POND_OK;
}

pond_status pond_mlp_set(pond_mlp *m, const float *params)
{
    if (!m || !params) return POND_EINVAL;
    return mlp_upload(m->dev, params, m->stream);
}

pond_status pond_mlp_forward(pond_mlp *m, const float *X, int64_t n, float *Y, void *stream)
{
    if (!m || !X || !Y || n < 0) return POND_EINVAL;
    hipStream_t st = stream ? (hipStream_t)stream : m->stream;
    if (n == 0) return POND_OK;
    unsigned grid = (unsigned)std::min<int64_t>((n + 15) / 16, 4096);
    mlp_forward_kernel<<<grid, 64, 0, st>>>(m->dev.wbf, m->dev.master, X, n, Y);
    HIPCHK(hipGetLastError());
    if (!stream) HIPCHK(hipStreamSynchronize(st));
    return POND_OK;
}

pond_status pond_mlp_grad(pond_mlp *m, const float *X, const float *T, int64_t n, float *grad, float *loss)
{
    if (!m || !X || !T || !grad || n < 1) return POND_EINVAL;
    int nw = train_grid(n, m->dev.npartial);
    mlp_train_kernel<<<nw, 64, 0, m->stream>>>(m->dev.wbf, m->dev.master, X, T, n, m->dev.partial);
    mlp_reduce_kernel<<<blocks(MLP_NPARAM + 1, 256), 256, 0, m->stream>>>(m->dev.partial, nw, m->dev.grad);
    HIPCHK(hipGetLastError());
    std::vector<float> h(MLP_NPARAM + 1);
    HIPCHK(hipMemcpyAsync(h.data(), m->dev.grad, sizeof(float) * (MLP_NPARAM + 1), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    std::copy(h.begin(), h.begin() + MLP_NPARAM, grad);
    if (loss) *loss = h[MLP_NPARAM];
    return POND_OK;
}

pond_status pond_mlp_train(pond_mlp *m, const float *X, const float *T, int64_t n, const pond_train_cfg *cfg,
                           float *loss_out)
{
    if (!train_args_ok(m, X, T, n, cfg)) return POND_EINVAL;
    MlpDevice &M = m->dev;
    const int64_t B = cfg->batch;
    std::vector<float> losses;
    for (int e = 0; e < cfg->epochs; ++e) {
        // each batch's loss lands in grad[NPARAM]; collected on the device side per batch
        std::vector<float> hl;
        float *dloss = nullptr;
        int64_t nbatches = (n + B - 1) / B;
        HIPCHK(hipMalloc(&dloss, sizeof(float) * nbatches));
        const int nb = train_epoch(M, X, T, n, cfg, m->stream, dloss);
        HIPCHK(hipGetLastError());
        hl.resize(nb);
        HIPCHK(hipMemcpyAsync(hl.data(), dloss, sizeof(float) * nb, hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        (void)hipFree(dloss);
        double sum = 0.0;
        for (float v : hl) sum += v;
        losses.push_back((float)(sum / std::max(nb, 1)));
    }
    if (loss_out) std::copy(losses.begin(), losses.end(), loss_out);
    return POND_OK;
}

pond_status pond_mlp_train_noalloc(pond_mlp *m, const float *X, const float *T, int64_t n,
                                   const pond_train_cfg *cfg, float *loss_out)
{
    if (!train_args_ok(m, X, T, n, cfg)) return POND_EINVAL;
    const int64_t nbatches = (n + cfg->batch - 1) / cfg->batch;
    if (nbatches > POND_NOALLOC_MAX_BATCHES || cfg->epochs > POND_NOALLOC_MAX_EPOCHS) {
        fprintf(stderr,
                "libpond: pond_mlp_train_noalloc: %lld batches per epoch and %d epochs, the static "
                "buffer holds at most %d and %d\n",
                (long long)nbatches, cfg->epochs, POND_NOALLOC_MAX_BATCHES, POND_NOALLOC_MAX_EPOCHS);
        return POND_EINVAL;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device) return POND_ESTATE;
    float *buf = noalloc_scratch(dev);
    if (!buf) return POND_EDEVICE;
    float *dloss = buf, *means = buf + POND_NOALLOC_MAX_BATCHES;
    for (int e = 0; e < cfg->epochs; ++e) {
        const int nb = train_epoch(m->dev, X, T, n, cfg, m->stream, dloss);
        loss_mean_kernel<<<1, 64, 0, m->stream>>>(dloss, nb, means + e);
    }
    HIPCHK(hipGetLastError());
    if (loss_out && cfg->epochs > 0)
        HIPCHK(hipMemcpyAsync(loss_out, means, sizeof(float) * cfg->epochs, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return POND_OK;
}

void pond_mlp_free(pond_mlp *m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    mlp_free(m->dev);
    if (m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

pond_status pond_mlp_features(pond_ctx *c, float *X, float *ref)
{
    if (!c || !X || !ref || c->D == 3) return POND_EINVAL;
    const int64_t nf = c->P.nface;
    if (c->D == 1) {
        if (c->precision == POND_FP64)
            mlp_features_kernel<1, double><<<blocks(nf, 128), 128, 0, c->stream>>>(c->P, state_of<double>(c), X, ref);
        else
            mlp_features_kernel<1, float><<<blocks(nf, 128), 128, 0, c->stream>>>(c->P, state_of<float>(c), X, ref);
    } else {
        if (c->precision == POND_FP64)
            mlp_features_kernel<2, double><<<blocks(nf, 128), 128, 0, c->stream>>>(c->P, state_of<double>(c), X, ref);
        else
            mlp_features_kernel<2, float><<<blocks(nf, 128), 128, 0, c->stream>>>(c->P, state_of<float>(c), X, ref);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return POND_OK;
}

pond_status pond_mlp_targets(pond_ctx *c, const float *X, const float *ref, float *T)
{
    if (!c || !X || !ref || !T || c->D == 3) return POND_EINVAL;
    const int64_t nf = c->P.nface;
    if (c->D == 1) {
        if (c->precision == POND_FP64)
            mlp_targets_kernel<1, double><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<double>(c), X, ref, T);
        else
            mlp_targets_kernel<1, float><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<float>(c), X, ref, T);
    } else {
        if (c->precision == POND_FP64)
            mlp_targets_kernel<2, double><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<double>(c), X, ref, T);
        else
            mlp_targets_kernel<2, float><<<blocks(nf, 256), 256, 0, c->stream>>>(c->P, state_of<float>(c), X, ref, T);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return POND_OK;
}

pond_status pond_load_mlp(pond_ctx *c, const pond_mlp *m, int32_t hard_iters)
{
    if (!c || !m || !m->dev.ready || hard_iters < 1 || c->D == 3 || c->layout != POND_LAYOUT_HERMITE)
        return POND_EINVAL;
    drop_graph(c);
    MlpDevice &M = c->mlp;
    if (!M.master) {
        pond_status s = mlp_alloc(M, 1);
        if (s != POND_OK) return s;
        if (hipMalloc(&M.list, sizeof(int) * NSLOT * slot_cap(c->P.nface)) != hipSuccess ||
            hipMalloc(&M.count, sizeof(int) * NSLOT) != hipSuccess) {
            mlp_free(M);
            return POND_ENOMEM;
        }
    }
    HIPCHK(hipStreamSynchronize(m->stream));
    HIPCHK(hipMemcpyAsync(M.master, m->dev.master, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, c->stream));
    mlp_pack_kernel<<<blocks(MLP_H * MLP_IN, 256), 256, 0, c->stream>>>(M.master, M.wbf);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    M.hard_iters = hard_iters;
    M.ready = true;
    return POND_OK;
}

} // extern "C"
