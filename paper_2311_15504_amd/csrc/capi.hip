// Host side of the C ABI declared in include/enomr.h: argument checks,
// workspace layout, kernel launches on the context's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <utility>
#include <vector>

#include "../../include/enomr.h"
#include "kernels.hpp"
#include "adjoint.hpp"

namespace enomr {
__constant__ double c_a[kPool][kMaxW];
__constant__ double c_wa[2][kPool][kMaxW];
__constant__ int c_candpool[10][kPool];
__constant__ double c_wrow[10][kRowsMax];
#ifdef ENOMR_PHASE_STAMPS
__device__ unsigned long long g_phase_stamps[kStampBlocks * kStampWaves * kStampPhases];
#endif

// Device memory of enomr_rhs_noalloc, the entry point that allocates nothing:
// the per-line alphas of one operator evaluation.  Each device the library
// runs on holds its own copy until the process ends.  Host code never uses
// this name as an address: enomr_create takes the device address with
// hipGetSymbolAddress, per context (a context belongs to one device).
constexpr size_t kScratchDoubles = 131072;   // 1 MiB
__device__ __align__(256) double scratch[kScratchDoubles];
}  // namespace enomr

using namespace enomr;

enum { PROF_SWEEP_X = 0, PROF_SWEEP_Y = 1, PROF_AUX = 2, PROF_CLASSES = 3 };

struct enomr_ctx {
    int device;
    hipStream_t stream;
    unsigned* status;   // device word, latched non-physical flag
    double* scratch;    // device address of enomr::scratch on this device
    // kernel timing (enomr_profile_start/stop): HIP event pairs per class
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[PROF_CLASSES];
    size_t used[PROF_CLASSES] = {0, 0, 0};
};

struct enomr_batch {
    enomr_ctx* ctx = nullptr;
    int nprob = 0;                 // 1D problems
    int nprob2 = 0;                // 2D problems
    int tf = 128;                  // faces per tile of the 1D kernel (autotuned)
    unsigned nblocks = 0;          // persistent workgroups of the 1D kernel
    unsigned nblocks2 = 0;         // workgroups of the largest 2D sweep launch
    int shape2 = 1;                // the 2D sweeps' tile shape: index into kB2Shapes (autotuned)
    double tune2_ms[3] = {0, 0, 0};// one-step times of the 2D tile shapes
    BatchProb* d_probs = nullptr;
    int* d_order = nullptr;
    BatchProb2* d_probs2 = nullptr;
    // 2D problems by order: group g holds d_list2[first .. first+count-1]
    // (longest first), and its sweep launches take the tile lists at
    // d_tiles2 + off[shape][dir] (tiles[shape][dir] entries; dir 0: x faces)
    struct Group2 {
        int R = 0, first = 0, count = 0;
        long off[3][2] = {}, tiles[3][2] = {};
    };
    std::vector<Group2> groups2;
    int* d_list2 = nullptr;
    int2* d_tiles2 = nullptr;
    int* d_queue = nullptr;        // [2]: work counters (the 1D kernel takes [0])
    BatchParams* d_params = nullptr;
    double* d_ws = nullptr;        // stage states (and 2D line buffers) of every problem
    hipStream_t cap = nullptr;     // capture stream of the 1D launch; it runs there beside the 2D steps
    hipStream_t cap2 = nullptr;    // capture stream of the 2D step
    std::vector<hipStream_t> br;   // the 2D step's branches, one per order
    std::vector<hipEvent_t> brev;
    hipEvent_t fork = nullptr, join = nullptr, fork2 = nullptr;
    hipGraph_t graph = nullptr, graph2 = nullptr;
    hipGraphExec_t exec = nullptr, exec2 = nullptr;
    double tune_ms[3] = {0, 0, 0}; // one-step times of the tile widths 64, 128, 256
};

namespace {

thread_local std::string g_err;

enomr_status fail(enomr_status st, const std::string& msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ENOMR_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int nvar(const enomr_problem& p)
{
    if (p.system == ENOMR_EULER) return p.ndim == 2 ? 4 : 3;
    return 1;
}

bool order_ok(int order) { return order >= 5 && order <= 17 && (order & 1); }

enomr_status check_problem(const enomr_problem* p)
{
    if (!p) return fail(ENOMR_EINVAL, "problem is NULL");
    if (!order_ok(p->order)) return fail(ENOMR_EORDER, "order must be odd in 5..17");
    const int r = (p->order + 1) / 2;
    if (p->ndim != 1 && p->ndim != 2) return fail(ENOMR_EINVAL, "ndim must be 1 or 2");
    if (p->system != ENOMR_ADVECTION && p->system != ENOMR_BURGERS && p->system != ENOMR_EULER)
        return fail(ENOMR_EINVAL, "unknown system");
    if (p->system != ENOMR_EULER && p->ndim != 1) return fail(ENOMR_EINVAL, "scalar laws are 1D only");
    if (p->nx < 2 * r + 1) return fail(ENOMR_EINVAL, "nx must be at least 2r+1");
    if (p->ndim == 1 && p->ny != 1) return fail(ENOMR_EINVAL, "ny must be 1 for ndim = 1");
    if (p->ndim == 2 && p->ny < 2 * r + 1) return fail(ENOMR_EINVAL, "ny must be at least 2r+1");
    if (!(p->hx > 0.0) || (p->ndim == 2 && !(p->hy > 0.0))) return fail(ENOMR_EINVAL, "spacing must be > 0");
    if ((p->bc_x != ENOMR_PERIODIC && p->bc_x != ENOMR_OUTFLOW) ||
        (p->ndim == 2 && p->bc_y != ENOMR_PERIODIC && p->bc_y != ENOMR_OUTFLOW))
        return fail(ENOMR_EINVAL, "unknown boundary condition");
    if (p->system == ENOMR_EULER && !(p->gamma > 1.0)) return fail(ENOMR_EINVAL, "gamma must be > 1");
    if (p->system != ENOMR_EULER && p->split != ENOMR_SPLIT_LF && p->split != ENOMR_SPLIT_NONE)
        return fail(ENOMR_EINVAL, "unknown split");
    if (p->nx > (1L << 31) || p->ny > (1L << 31)) return fail(ENOMR_EINVAL, "grid too large");
    // 2D launch shapes: the alpha pass has ceil(ny/32) rows of workgroups (at
    // most 65535), and the sweeps' workgroup counts stay below 2^32 for
    // nx*ny <= 2^32 cells
    if (p->ndim == 2 && (p->ny > 65535L * 32 || p->nx * p->ny > (1L << 32)))
        return fail(ENOMR_EINVAL, "2D grid too large (ny <= 2097120, nx*ny <= 2^32)");
    if (p->recon != ENOMR_CHARACTERISTIC && p->recon != ENOMR_COMPONENTWISE)
        return fail(ENOMR_EINVAL, "unknown recon");
    if (p->alpha_mode != ENOMR_ALPHA_LINE && p->alpha_mode != ENOMR_ALPHA_FIELD)
        return fail(ENOMR_EINVAL, "unknown alpha_mode");
    if (p->system != ENOMR_EULER && (p->recon != ENOMR_CHARACTERISTIC || p->alpha_mode != ENOMR_ALPHA_LINE))
        return fail(ENOMR_EINVAL, "recon and alpha_mode apply to Euler problems");
    if (p->recon == ENOMR_COMPONENTWISE && p->alpha_mode == ENOMR_ALPHA_FIELD)
        return fail(ENOMR_EINVAL, "per-field alphas need the characteristic reconstruction");
    if (!std::isfinite(p->gravity)) return fail(ENOMR_EINVAL, "gravity must be finite");
    if (p->gravity != 0.0 && !(p->system == ENOMR_EULER && p->ndim == 2))
        return fail(ENOMR_EINVAL, "the gravity source applies to 2D Euler problems");
    return ENOMR_OK;
}

// The operator as the paper runs it (no variant switch set).
bool default_operator(const enomr_problem& p)
{
    return p.recon == ENOMR_CHARACTERISTIC && p.alpha_mode == ENOMR_ALPHA_LINE && p.gravity == 0.0;
}

int variant(const enomr_problem& p)
{
    if (p.recon == ENOMR_COMPONENTWISE) return VAR_COMPONENT;
    return p.alpha_mode == ENOMR_ALPHA_FIELD ? VAR_FIELD : VAR_CHAR;
}

// Workspace: two stage states, one operator buffer, per-line alphas and a
// few device scalars.
struct Layout {
    size_t U1, U2, L, ax, ay, ax2, ay2, dt, t, active, adj_tmp, total;
};

Layout layout(const enomr_problem& p)
{
    Layout w;
    const size_t state = sizeof(double) * nvar(p) * (size_t)p.nx * (size_t)p.ny;
    size_t off = 0;
    w.U1 = off; off += align_up(state);
    w.U2 = off; off += align_up(state);
    w.L = off; off += p.ndim == 2 ? align_up(state) : 0;
    // per-line alphas: three planes with per-field alphas
    const size_t na = p.alpha_mode == ENOMR_ALPHA_FIELD ? 3 : 1;
    w.ax = off; off += align_up(sizeof(double) * na * (size_t)p.ny);
    w.ay = off; off += align_up(sizeof(double) * na * (size_t)(p.ndim == 2 ? p.nx : 1));
    // a second set: the stages of a run alternate between the two
    w.ax2 = off; off += align_up(sizeof(double) * na * (size_t)p.ny);
    w.ay2 = off; off += align_up(sizeof(double) * na * (size_t)(p.ndim == 2 ? p.nx : 1));
    w.dt = off; off += 256;
    w.t = off; off += 256;
    w.active = off; off += 256;
    // frozen-stencil adjoint (1D Euler): three state-sized temporaries
    const bool adj = p.system == ENOMR_EULER && p.ndim == 1;
    w.adj_tmp = off; off += adj ? 3 * align_up(state) : 0;
    w.total = off;
    return w;
}

template <typename T>
T* at(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

unsigned blocks_for(long n, int per) { return (unsigned)((n + per - 1) / per); }

// Bracket a launch with HIP events of class `cls` when profiling is on.
template <typename F>
void timed(enomr_ctx* ctx, int cls, F&& launch)
{
    if (!ctx->prof) {
        launch();
        return;
    }
    auto& v = ctx->ev[cls];
    if (ctx->used[cls] == v.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            launch();
            return;
        }
        v.emplace_back(a, b);
    }
    auto& pr = v[ctx->used[cls]++];
    (void)hipEventRecord(pr.first, ctx->stream);
    launch();
    (void)hipEventRecord(pr.second, ctx->stream);
}

#define DISPATCH_R(order, ...)                      \
    switch (((order) + 1) / 2) {                    \
    case 3: { constexpr int R = 3; __VA_ARGS__; } break;  \
    case 4: { constexpr int R = 4; __VA_ARGS__; } break;  \
    case 5: { constexpr int R = 5; __VA_ARGS__; } break;  \
    case 6: { constexpr int R = 6; __VA_ARGS__; } break;  \
    case 7: { constexpr int R = 7; __VA_ARGS__; } break;  \
    case 8: { constexpr int R = 8; __VA_ARGS__; } break;  \
    case 9: { constexpr int R = 9; __VA_ARGS__; } break;  \
    default: break;                                 \
    }

#define DISPATCH_VAR(var, ...)                                                     \
    switch (var) {                                                                 \
    case VAR_COMPONENT: { constexpr int V = VAR_COMPONENT; __VA_ARGS__; } break;   \
    case VAR_FIELD: { constexpr int V = VAR_FIELD; __VA_ARGS__; } break;           \
    default: { constexpr int V = VAR_CHAR; __VA_ARGS__; } break;                   \
    }

// Tile shapes (faces per line x lines per block).
constexpr int kTF1 = 64;                  // 1D lines
// Scalar laws: windows shared lane to lane (k_scalar_sweep_dpp) or staged in
// LDS (k_scalar_sweep), per order by measurement on MI355X (1D advection,
// 2^27 nodes): lane sharing is 1% faster at order 5 and slower from order 7
// up, where its register windows (4 cells per lane) lower the occupancy to
// 2-4 waves per SIMD.
constexpr bool scalar_lane_shared(int R) { return R == 3; }
constexpr int kMaxLsspStages = 18;        // linear SSP-RK(m, m-1): m up to order 17 + 1
constexpr int kTFx = 64, kTLx = 4;        // 2D x sweep
constexpr int kTFy = 64, kTLy = 4;        // 2D y sweep

// Where the per-line alphas of one operator evaluation live: ay follows ax,
// so one fill of nfill doubles from ax clears both (and the padding between).
struct AlphaBufs {
    double* ax;
    double* ay;
    long nfill;
};

long alpha_count_x(const enomr_problem& p) { return (p.alpha_mode == ENOMR_ALPHA_FIELD ? 3 : 1) * (long)p.ny; }
long alpha_count_y(const enomr_problem& p)
{
    return (p.alpha_mode == ENOMR_ALPHA_FIELD ? 3 : 1) * (long)(p.ndim == 2 ? p.nx : 1);
}

AlphaBufs alpha_bufs(const enomr_problem& p, void* ws)
{
    const Layout w = layout(p);
    return AlphaBufs{at<double>(ws, w.ax), at<double>(ws, w.ay),
                     (long)(w.ay - w.ax) / (long)sizeof(double) + alpha_count_y(p)};
}

// Alpha set k % 2 of a run's stages (set 0 is the one alpha_bufs gives).
AlphaBufs alpha_bufs_run(const enomr_problem& p, void* ws, long k)
{
    if (k % 2 == 0) return alpha_bufs(p, ws);
    const Layout w = layout(p);
    return AlphaBufs{at<double>(ws, w.ax2), at<double>(ws, w.ay2),
                     (long)(w.ay2 - w.ax2) / (long)sizeof(double) + alpha_count_y(p)};
}

// The same two arrays packed from `base` (256-byte aligned), for
// enomr_rhs_noalloc; doubles_needed() is their extent.
long alpha_ax_extent(const enomr_problem& p) { return (alpha_count_x(p) + 31) & ~31L; }
long doubles_needed(const enomr_problem& p) { return alpha_ax_extent(p) + alpha_count_y(p); }
AlphaBufs alpha_bufs_at(const enomr_problem& p, double* base)
{
    return AlphaBufs{base, base + alpha_ax_extent(p), doubles_needed(p)};
}

// Alphas of every line of `Us` into ab (zeroed first).  With `next` (Euler
// only), ab already holds zeros and the alpha kernel zeroes `next`, the
// buffer of the run's following stage, instead of a fill launch.
enomr_status launch_alpha(enomr_ctx* ctx, const enomr_problem& p, const double* Us, const AlphaBufs& ab,
                          const int* active, const AlphaBufs* next = nullptr)
{
    double* ax = ab.ax;
    double* ay = ab.ay;
    const bool pf = p.alpha_mode == ENOMR_ALPHA_FIELD;
    timed(ctx, PROF_AUX, [&] {
        const long nfill = ab.nfill;
        double* zp = nullptr;
        long zn = 0;
        if (next && p.system == ENOMR_EULER) {
            zp = next->ax;
            zn = next->nfill;
        } else {
            hipLaunchKernelGGL(k_fill, dim3(blocks_for(nfill, 256)), dim3(256), 0, ctx->stream, ax, nfill, 0.0);
        }
        if (p.system == ENOMR_EULER) {
            dim3 grid(blocks_for(p.nx, 64), blocks_for(p.ny, 32));
            if (pf && p.ndim == 2)
                hipLaunchKernelGGL((k_alpha_euler<4, true>), grid, dim3(256), 0, ctx->stream, Us, (long)p.nx,
                                   (long)p.ny, p.gamma, ax, ay, ctx->status, active, zp, zn);
            else if (pf)
                hipLaunchKernelGGL((k_alpha_euler<3, true>), grid, dim3(256), 0, ctx->stream, Us, (long)p.nx,
                                   (long)p.ny, p.gamma, ax, ay, ctx->status, active, zp, zn);
            else if (p.ndim == 2)
                hipLaunchKernelGGL(k_alpha_euler<4>, grid, dim3(256), 0, ctx->stream, Us, (long)p.nx, (long)p.ny,
                                   p.gamma, ax, ay, ctx->status, active, zp, zn);
            else
                hipLaunchKernelGGL(k_alpha_euler<3>, grid, dim3(256), 0, ctx->stream, Us, (long)p.nx, (long)p.ny,
                                   p.gamma, ax, ay, ctx->status, active, zp, zn);
        } else {
            // a few thousand workgroups of eight cells per thread (a pass over
            // the line for Burgers; advection needs none)
            const unsigned nb = blocks_for(p.nx, 256 * 8) < 2048 ? blocks_for(p.nx, 256 * 8) : 2048;
            hipLaunchKernelGGL(k_alpha_scalar, dim3(nb), dim3(256), 0, ctx->stream, Us, (long)p.nx,
                               p.system == ENOMR_ADVECTION ? SYS_ADVECTION : SYS_BURGERS, p.adv_speed, ax, active);
        }
    });
    HIP_TRY(hipGetLastError());
    return ENOMR_OK;
}

enomr_status launch_alpha(enomr_ctx* ctx, const enomr_problem& p, const double* Us, void* ws, const int* active)
{
    return launch_alpha(ctx, p, Us, alpha_bufs(p, ws), active);
}

// The operator L(Us) and its use: stage 0 stores L into so.out, stages 1..3
// combine the SSP-RK3 stage.  Requires the alphas of Us in ab.  2D: the y
// sweep stores L_y into Ly, which the x sweep reads back cell by cell (each
// thread reads and writes only its own cells, so Ly may be so.out).
enomr_status launch_operator(enomr_ctx* ctx, const enomr_problem& p, const double* Us, StageOut so,
                             uint8_t* idx, const AlphaBufs& ab, double* Ly, const int* active)
{
    const double* ax = ab.ax;
    const double* ay = ab.ay;
    if (p.system != ENOMR_EULER) {
        const int flux = p.system == ENOMR_ADVECTION ? SYS_ADVECTION : SYS_BURGERS;
        const int split = p.split == ENOMR_SPLIT_LF ? 1 : 0;
        timed(ctx, PROF_SWEEP_X, [&] {
            DISPATCH_R(p.order,
                       if constexpr (scalar_lane_shared(R)) {
                           // DppTile<R>::CW cells per wave, four waves per block
                           const long nw = (long)blocks_for(p.nx, DppTile<R>::CW);
                           hipLaunchKernelGGL((k_scalar_sweep_dpp<R>), dim3(blocks_for(nw, 4)), dim3(256), 0,
                                              ctx->stream, Us, (long)p.nx, 1.0 / p.hx, flux, p.adv_speed, split,
                                              p.bc_x, ax, so, idx, active);
                       } else {
                           hipLaunchKernelGGL((k_scalar_sweep<R, kTF1>), dim3(blocks_for(p.nx, kTF1 - 1)),
                                              dim3(kTF1), 0, ctx->stream, Us, (long)p.nx, 1.0 / p.hx, flux,
                                              p.adv_speed, split, p.bc_x, ax, so, idx, active);
                       });
        });
        HIP_TRY(hipGetLastError());
        return ENOMR_OK;
    }
    SweepIn in;
    in.Us = Us;
    in.status = ctx->status;
    in.active = active;
    in.nx = p.nx;
    in.ny = p.ny;
    in.gamma = p.gamma;
    in.grav = 0.0;
    const int var = variant(p);
    if (p.ndim == 1) {
        in.alpha = ax;
        in.idx = idx;
        in.ih = 1.0 / p.hx;
        in.bc = p.bc_x;
        timed(ctx, PROF_SWEEP_X, [&] {
            DISPATCH_VAR(var, DISPATCH_R(p.order,
                       hipLaunchKernelGGL((k_euler_sweep<3, R, 0, kTF1, 1, V>), dim3(blocks_for(p.nx, kTF1 - 1)),
                                          dim3(kTF1), 0, ctx->stream, in, so)));
        });
        HIP_TRY(hipGetLastError());
        return ENOMR_OK;
    }
    // 2D: the y sweep stores L_y, then the x sweep adds L_x (L_y + L_x =
    // L_x + L_y exactly) and the source, and either stores the sum or combines
    // the RK stage: the output phase with its extra reads runs in the sweep
    // whose lines are rows, so those reads are coalesced.
    StageOut sy;
    sy.Un = nullptr;
    sy.Lprev = nullptr;
    sy.out = Ly;
    sy.dt = nullptr;
    sy.stage = 0;
    in.alpha = ay;
    in.idx = idx ? idx + (size_t)p.ny * (p.nx + 1) * 8 : nullptr;
    in.ih = 1.0 / p.hy;
    in.bc = p.bc_y;
    in.grav = 0.0;
    timed(ctx, PROF_SWEEP_Y, [&] {
        DISPATCH_VAR(var, DISPATCH_R(p.order,
                   hipLaunchKernelGGL((k_euler_sweep<4, R, 1, kTFy, kTLy, V>),
                                      dim3(blocks_for(p.ny, kTFy - 1) * blocks_for(p.nx, kTLy)), dim3(kTFy * kTLy),
                                      0, ctx->stream, in, sy)));
    });
    HIP_TRY(hipGetLastError());
    in.alpha = ax;
    in.idx = idx;
    in.ih = 1.0 / p.hx;
    in.bc = p.bc_x;
    in.grav = p.gravity;
    so.Lprev = Ly;
    timed(ctx, PROF_SWEEP_X, [&] {
        DISPATCH_VAR(var, DISPATCH_R(p.order,
                   hipLaunchKernelGGL((k_euler_sweep<4, R, 0, kTFx, kTLx, V>),
                                      dim3(blocks_for(p.nx, kTFx - 1) * blocks_for(p.ny, kTLx)), dim3(kTFx * kTLx),
                                      0, ctx->stream, in, so)));
    });
    HIP_TRY(hipGetLastError());
    return ENOMR_OK;
}

enomr_status launch_operator(enomr_ctx* ctx, const enomr_problem& p, const double* Us, StageOut so,
                             uint8_t* idx, void* ws, const int* active)
{
    return launch_operator(ctx, p, Us, so, idx, alpha_bufs(p, ws), at<double>(ws, layout(p).L), active);
}

size_t idx_bytes(const enomr_problem& p)
{
    if (p.system != ENOMR_EULER) return (size_t)(p.nx + 1) * 2;
    if (p.ndim == 1) return (size_t)(p.nx + 1) * 6;
    return (size_t)p.ny * (p.nx + 1) * 8 + (size_t)(p.ny + 1) * p.nx * 8;
}

enomr_status launch_dt(enomr_ctx* ctx, const enomr_problem& p, double cfl, void* ws, const AlphaBufs& ab,
                       double* dt, double t_end, double* dt_log, long step)
{
    const Layout w = layout(p);
    // per-field alphas: the maximum over the three planes is max(|u|+c)
    const long na = p.alpha_mode == ENOMR_ALPHA_FIELD ? 3 : 1;
    const long nax = p.system == ENOMR_EULER ? na * p.ny : 1;
    const long nay = p.ndim == 2 ? na * p.nx : 0;
    timed(ctx, PROF_AUX, [&] {
        hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, ctx->stream, ab.ax, nax, ab.ay, nay, cfl, 1.0 / p.hx,
                           p.ndim == 2 ? 1.0 / p.hy : 0.0, t_end, dt, at<double>(ws, w.t), at<int>(ws, w.active),
                           dt_log, step);
    });
    HIP_TRY(hipGetLastError());
    return ENOMR_OK;
}

// One SSP-RK3 step of U in place.  With run (the count of the run's stages
// so far), stage k takes alpha set k % 2, whose zeros the previous stage's
// alpha launch wrote, and its own alpha launch zeroes the other set;
// alpha_ready: the first stage's alphas (and dt) are already in place.
// Without run, every stage fills set 0 before its alpha launch.
enomr_status rk3_step(enomr_ctx* ctx, const enomr_problem& p, double* U, const double* dt, void* ws,
                      uint8_t* idx_log, const int* active, bool alpha_ready, long* run = nullptr)
{
    const Layout w = layout(p);
    double* U1 = at<double>(ws, w.U1);
    double* U2 = at<double>(ws, w.U2);
    const double* stage_in[3] = {U, U1, U2};
    double* stage_out[3] = {U1, U2, U};
    const size_t ib = idx_bytes(p);
    for (int s = 0; s < 3; ++s) {
        const AlphaBufs ab = run ? alpha_bufs_run(p, ws, *run) : alpha_bufs(p, ws);
        if (!(s == 0 && alpha_ready)) {
            const AlphaBufs next = alpha_bufs_run(p, ws, run ? *run + 1 : 1);
            enomr_status st = launch_alpha(ctx, p, stage_in[s], ab, active, run ? &next : nullptr);
            if (st) return st;
        }
        StageOut so;
        so.Un = U;
        so.Lprev = nullptr;
        so.out = stage_out[s];
        so.dt = dt;
        so.stage = s + 1;
        enomr_status st = launch_operator(ctx, p, stage_in[s], so, idx_log ? idx_log + s * ib : nullptr, ab,
                                          at<double>(ws, w.L), active);
        if (st) return st;
        if (run) ++*run;
    }
    return ENOMR_OK;
}

// One reverse stage of the frozen 1D Euler operator (see AdjIn): one launch,
// kAdjT cells per workgroup.
constexpr int kAdjT = 32, kAdjNT = 128;

enomr_status launch_adjoint_stage(enomr_ctx* ctx, const enomr_problem& p, AdjIn a)
{
    a.status = ctx->status;
    a.n = p.nx;
    a.ih = 1.0 / p.hx;
    a.gamma = p.gamma;
    a.bc = p.bc_x;
    DISPATCH_R(p.order, hipLaunchKernelGGL((k_adj_stage<R, kAdjT, kAdjNT>), dim3(blocks_for(p.nx, kAdjT)),
                                          dim3(kAdjNT), 0, ctx->stream, a));
    HIP_TRY(hipGetLastError());
    return ENOMR_OK;
}

// Forward steps recording what the reverse sweep needs (see the header).
enomr_status record_steps(enomr_ctx* ctx, const enomr_problem& p, double* U, double cfl, int64_t nsteps,
                          double* stages, uint8_t* idx_log, double* alpha_log, double* dt_log, void* ws)
{
    const size_t ns = (size_t)3 * p.nx;
    const size_t ib = idx_bytes(p);
    // alternating alpha sets, as in enomr_advance: one fill for the run
    long run = 0;
    if (nsteps > 0) {
        const AlphaBufs a0 = alpha_bufs_run(p, ws, 0);
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(a0.nfill, 256)), dim3(256), 0, ctx->stream, a0.ax, a0.nfill, 0.0);
        HIP_TRY(hipGetLastError());
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        double* S[3] = {stages + (3 * k) * ns, stages + (3 * k + 1) * ns, stages + (3 * k + 2) * ns};
        uint8_t* ix = idx_log + (size_t)k * 3 * ib;
        double* al = alpha_log + 3 * k;
        double* dt = dt_log + k;
        HIP_TRY(hipMemcpyAsync(S[0], U, sizeof(double) * ns, hipMemcpyDeviceToDevice, ctx->stream));
        double* outs[3] = {S[1], S[2], U};
        for (int s = 0; s < 3; ++s, ++run) {
            const AlphaBufs ab = alpha_bufs_run(p, ws, run);
            const AlphaBufs next = alpha_bufs_run(p, ws, run + 1);
            if (enomr_status st = launch_alpha(ctx, p, S[s], ab, nullptr, &next)) return st;
            hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, ctx->stream, al + s, ab.ax);
            HIP_TRY(hipGetLastError());
            if (s == 0)
                if (enomr_status st = launch_dt(ctx, p, cfl, ws, ab, dt, 0.0, nullptr, 0)) return st;
            StageOut so;
            so.Un = S[0];
            so.Lprev = nullptr;
            so.out = outs[s];
            so.dt = dt;
            so.stage = s + 1;
            if (enomr_status st = launch_operator(ctx, p, S[s], so, ix + s * ib, ab, at<double>(ws, layout(p).L),
                                                  nullptr))
                return st;
        }
    }
    return ENOMR_OK;
}

// Reverse sweep over recorded steps, last step first; lam in place.
enomr_status adjoint_steps(enomr_ctx* ctx, const enomr_problem& p, int64_t nsteps, const double* stages,
                           const uint8_t* idx_log, const double* alpha_log, const double* dt_log, double* lam,
                           void* ws)
{
    const Layout w = layout(p);
    const size_t ns = (size_t)3 * p.nx;
    const size_t ib = idx_bytes(p);
    const size_t sb = align_up(sizeof(double) * ns);
    double* T1 = at<double>(ws, w.adj_tmp);        // adjoint of U^(2)
    double* T2 = at<double>(ws, w.adj_tmp + sb);   // adjoint of U^(1)
    double* T4 = at<double>(ws, w.adj_tmp + 2 * sb);   // adjoint of U^n (partial)
    const double c13 = 1.0 / 3.0, c23 = 2.0 / 3.0;
    for (int64_t k = nsteps - 1; k >= 0; --k) {
        const double* S[3] = {stages + (3 * k) * ns, stages + (3 * k + 1) * ns, stages + (3 * k + 2) * ns};
        const uint8_t* ix = idx_log + (size_t)k * 3 * ib;
        const double* al = alpha_log + 3 * k;
        const double* dt = dt_log + k;
        AdjIn a{};
        a.dt = dt;
        // stage 3: U^{n+1} = 1/3 U^n + 2/3 (U^(2) + dt L(U^(2)))
        a.U = S[2]; a.idx = ix + 2 * ib; a.alpha = al + 2; a.lamIn = lam;
        a.a = c13; a.b = c23; a.cb = c23; a.addv = nullptr; a.lamAcc = T4; a.accumulate = 0; a.lamOut = T1;
        if (enomr_status st = launch_adjoint_stage(ctx, p, a)) return st;
        // stage 2: U^(2) = 3/4 U^n + 1/4 (U^(1) + dt L(U^(1)))
        a.U = S[1]; a.idx = ix + ib; a.alpha = al + 1; a.lamIn = T1;
        a.a = 0.75; a.b = 0.25; a.cb = 0.25; a.addv = nullptr; a.lamAcc = T4; a.accumulate = 1; a.lamOut = T2;
        if (enomr_status st = launch_adjoint_stage(ctx, p, a)) return st;
        // stage 1: U^(1) = U^n + dt L(U^n)
        a.U = S[0]; a.idx = ix; a.alpha = al; a.lamIn = T2;
        a.a = 0.0; a.b = 1.0; a.cb = 1.0; a.addv = T4; a.lamAcc = nullptr; a.accumulate = 0; a.lamOut = lam;
        if (enomr_status st = launch_adjoint_stage(ctx, p, a)) return st;
    }
    return ENOMR_OK;
}

enomr_status check_adjoint_problem(const enomr_problem* p)
{
    if (enomr_status st = check_problem(p)) return st;
    if (p->system != ENOMR_EULER || p->ndim != 1)
        return fail(ENOMR_EINVAL, "the adjoint is provided for 1D Euler problems");
    if (!default_operator(*p)) return fail(ENOMR_EINVAL, "the adjoint takes the default operator only");
    return ENOMR_OK;
}

enomr_status check_ctx(enomr_ctx* ctx)
{
    if (!ctx) return fail(ENOMR_EINVAL, "context is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(ENOMR_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    return ENOMR_OK;
}

}  // namespace

extern "C" {

const char* enomr_last_error(void) { return g_err.c_str(); }

enomr_status enomr_coefficients(int order, int32_t* ncand, int32_t* mn, double* a, double* b)
{
    if (!order_ok(order)) return fail(ENOMR_EORDER, "order must be odd in 5..17");
    static double ta[kPool][kMaxW], tb[kPool][kMaxW];
    static bool ready = generate_tables(ta, tb);
    (void)ready;
    const int R = (order + 1) / 2;
    const int nc = n_cands(R);
    if (ncand) *ncand = nc;
    for (int c = 0; c < nc; ++c) {
        const int P = cand_pool(R, c);
        if (mn) {
            mn[2 * c] = pool_mn(P, 0);
            mn[2 * c + 1] = pool_mn(P, 1);
        }
        for (int l = 0; l < kMaxW; ++l) {
            if (a) a[c * kMaxW + l] = ta[P][l];
            if (b) b[c * kMaxW + l] = tb[P][l];
        }
    }
    return ENOMR_OK;
}

enomr_status enomr_create(int device, void* hip_stream, enomr_ctx** out)
{
    if (!out) return fail(ENOMR_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(ENOMR_ENODEV, "no such device");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(ENOMR_ENODEV, std::string("library built for gfx950, device is ") + prop.gcnArchName);
    static double ta[kPool][kMaxW], tb[kPool][kMaxW];
    static bool ready = generate_tables(ta, tb);
    (void)ready;
    // window-aligned rows (centre at entry 8) and candidate -> pool maps
    static double wa[2][kPool][kMaxW];
    static int cp[10][kPool];
    for (int P = 0; P < kPool; ++P) {
        const int m = pool_mn(P, 0), n = pool_mn(P, 1);
        for (int i = 0; i < kMaxW; ++i) {
            wa[0][P][i] = wa[1][P][i] = 0.0;
        }
        for (int l = -m; l <= n; ++l) {
            wa[0][P][8 + l] = ta[P][l + m];   // f^+: offset l is window entry 8 + l
            wa[1][P][8 - l] = ta[P][l + m];   // f^-: offset l is window entry 8 - l
        }
    }
    for (int R = 0; R < 10; ++R)
        for (int c = 0; c < kPool; ++c) cp[R][c] = (R >= 3 && c < n_cands(R)) ? cand_pool(R, c) : 0;
    HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_a), ta, sizeof(ta)));
    HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_wa), wa, sizeof(wa)));
    HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_candpool), cp, sizeof(cp)));
    // the f^+ window rows of candidates 1 .. n_cands(R)-4, per order
    static double wr[10][kRowsMax];
    for (int R = 0; R < 10; ++R) {
        for (int e = 0; e < kRowsMax; ++e) wr[R][e] = 0.0;
        if (R < 3) continue;
        const int W = 2 * R - 1;
        for (int c = 1; c <= n_cands(R) - 4; ++c)
            for (int i = 0; i < W; ++i) wr[R][(c - 1) * W + i] = wa[0][cp[R][c]][9 - R + i];
    }
    HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_wrow), wr, sizeof(wr)));
    // this device's copy of the scratch array of enomr_rhs_noalloc
    void* scratch_addr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&scratch_addr, HIP_SYMBOL(enomr::scratch)));
    enomr_ctx* c = new enomr_ctx;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->status = nullptr;
    c->scratch = static_cast<double*>(scratch_addr);
    hipError_t e = hipMalloc(&c->status, sizeof(unsigned));
    if (e != hipSuccess) {
        delete c;
        return fail(ENOMR_ENOMEM, "cannot allocate the status word");
    }
    e = hipMemset(c->status, 0, sizeof(unsigned));
    if (e != hipSuccess) {
        (void)hipFree(c->status);
        delete c;
        return fail(ENOMR_EHIP, "cannot clear the status word");
    }
    *out = c;
    return ENOMR_OK;
}

enomr_status enomr_destroy(enomr_ctx* ctx)
{
    if (!ctx) return ENOMR_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipFree(ctx->status);
    for (auto& v : ctx->ev)
        for (auto& pr : v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    delete ctx;
    return ENOMR_OK;
}

enomr_status enomr_set_stream(enomr_ctx* ctx, void* hip_stream)
{
    if (!ctx) return fail(ENOMR_EINVAL, "context is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return ENOMR_OK;
}

enomr_status enomr_recon_faces(enomr_ctx* ctx, int order, int sign, int64_t n, const double* f_with_halo,
                               double* fhat, uint8_t* idx)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (!order_ok(order)) return fail(ENOMR_EORDER, "order must be odd in 5..17");
    if (sign != 1 && sign != -1) return fail(ENOMR_EINVAL, "sign must be +1 or -1");
    if (n < 0 || (n > 0 && (!f_with_halo || !fhat))) return fail(ENOMR_EINVAL, "bad arrays");
    if (n > (int64_t(1) << 38)) return fail(ENOMR_EINVAL, "n too large (at most 2^38 faces)");   // grid < 2^32 blocks
    if (n == 0) return ENOMR_OK;
    const unsigned nb = blocks_for(n, 256);
    if (sign > 0) {
        DISPATCH_R(order, hipLaunchKernelGGL((k_recon_faces<R, 1>), dim3(nb), dim3(256), 0, ctx->stream,
                                             f_with_halo, (long)n, fhat, idx));
    } else {
        DISPATCH_R(order, hipLaunchKernelGGL((k_recon_faces<R, -1>), dim3(nb), dim3(256), 0, ctx->stream,
                                             f_with_halo, (long)n, fhat, idx));
    }
    HIP_TRY(hipGetLastError());
    return ENOMR_OK;
}

enomr_status enomr_workspace_size(const enomr_problem* prob, size_t* bytes)
{
    if (enomr_status st = check_problem(prob)) return st;
    if (!bytes) return fail(ENOMR_EINVAL, "bytes is NULL");
    *bytes = layout(*prob).total;
    return ENOMR_OK;
}

enomr_status enomr_rhs(enomr_ctx* ctx, const enomr_problem* prob, const double* U, double* dUdt, uint8_t* idx,
                       void* ws)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_problem(prob)) return st;
    if (!U || !dUdt || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (enomr_status st = launch_alpha(ctx, *prob, U, ws, nullptr)) return st;
    StageOut so;
    so.Un = nullptr;
    so.Lprev = nullptr;
    so.out = dUdt;
    so.dt = nullptr;
    so.stage = 0;
    return launch_operator(ctx, *prob, U, so, idx, ws, nullptr);
}

enomr_status enomr_rhs_noalloc(enomr_ctx* ctx, const enomr_problem* prob, const double* U, double* dUdt,
                               uint8_t* idx)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_problem(prob)) return st;
    if (!U || !dUdt) return fail(ENOMR_EINVAL, "NULL array");
    if (U == dUdt) return fail(ENOMR_EINVAL, "dUdt must not alias U");
    if (!ctx->scratch) return fail(ENOMR_EHIP, "the scratch array has no device address");
    const long need = doubles_needed(*prob);
    if (need > (long)kScratchDoubles)
        return fail(ENOMR_EINVAL, "enomr_rhs_noalloc: the problem's per-line alphas need " + std::to_string(need) +
                                      " doubles of scratch; at most " + std::to_string(kScratchDoubles) +
                                      " are available (use enomr_rhs with a workspace)");
    const AlphaBufs ab = alpha_bufs_at(*prob, ctx->scratch);
    if (enomr_status st = launch_alpha(ctx, *prob, U, ab, nullptr)) return st;
    StageOut so;
    so.Un = nullptr;
    so.Lprev = nullptr;
    so.out = dUdt;
    so.dt = nullptr;
    so.stage = 0;
    // 2D: L_y goes through dUdt itself
    return launch_operator(ctx, *prob, U, so, idx, ab, dUdt, nullptr);
}

enomr_status enomr_dt(enomr_ctx* ctx, const enomr_problem* prob, const double* U, double cfl, double* dt_dev,
                      void* ws)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_problem(prob)) return st;
    if (!U || !dt_dev || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (!(cfl > 0.0)) return fail(ENOMR_EINVAL, "cfl must be > 0");
    if (enomr_status st = launch_alpha(ctx, *prob, U, ws, nullptr)) return st;
    return launch_dt(ctx, *prob, cfl, ws, alpha_bufs(*prob, ws), dt_dev, 0.0, nullptr, 0);
}

enomr_status enomr_ssprk3_step(enomr_ctx* ctx, const enomr_problem* prob, double* U, const double* dt_dev,
                               void* ws, uint8_t* idx_log)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_problem(prob)) return st;
    if (!U || !dt_dev || !ws) return fail(ENOMR_EINVAL, "NULL array");
    return rk3_step(ctx, *prob, U, dt_dev, ws, idx_log, nullptr, false);
}

enomr_status enomr_advance(enomr_ctx* ctx, const enomr_problem* prob, double* U, double cfl, int64_t nsteps,
                           double t_end, void* ws, double* dt_log)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_problem(prob)) return st;
    if (!U || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (!(cfl > 0.0) || nsteps < 0) return fail(ENOMR_EINVAL, "bad cfl or nsteps");
    const Layout w = layout(*prob);
    double* dt = at<double>(ws, w.dt);
    int* active = at<int>(ws, w.active);
    double* t = at<double>(ws, w.t);
    // t = 0, active = 1 (fill kernels, so a captured sequence replays cleanly)
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, ctx->stream, t, 1L, 0.0);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, ctx->stream, active, 1);
    HIP_TRY(hipGetLastError());
    const int* act = t_end > 0.0 ? active : nullptr;
    // the stages alternate between the two alpha sets: each stage's alpha
    // launch zeroes the next stage's set, so only the first needs a fill
    long run = 0;
    const bool euler = prob->system == ENOMR_EULER;
    if (euler && nsteps > 0) {
        const AlphaBufs a0 = alpha_bufs_run(*prob, ws, 0);
        hipLaunchKernelGGL(k_fill, dim3(blocks_for(a0.nfill, 256)), dim3(256), 0, ctx->stream, a0.ax, a0.nfill, 0.0);
        HIP_TRY(hipGetLastError());
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        const AlphaBufs ab = alpha_bufs_run(*prob, ws, run);
        const AlphaBufs next = alpha_bufs_run(*prob, ws, run + 1);
        if (enomr_status st = launch_alpha(ctx, *prob, U, ab, act, euler ? &next : nullptr)) return st;
        if (enomr_status st = launch_dt(ctx, *prob, cfl, ws, ab, dt, t_end, dt_log, (long)s)) return st;
        if (enomr_status st = rk3_step(ctx, *prob, U, dt, ws, nullptr, act, true, euler ? &run : nullptr)) return st;
    }
    return ENOMR_OK;
}

// ---------------------------------------------------------------------------
// Linear SSP-RK(m, m-1) (Sec. 2.3, Eqs. lSSPRK, lSSPRK_Coe) for scalar lines
// ---------------------------------------------------------------------------

namespace {

// alpha_{m,0..m-1} in exact rationals, rounded to the nearest doubles:
// alpha_{2,0} = 0, alpha_{2,1} = 1; alpha_{m,k} = (2/k) alpha_{m-1,k-1} for
// 1 <= k <= m-2; alpha_{m,m-1} = (2/m) alpha_{m-1,m-2};
// alpha_{m,0} = 1 - sum_{k>=1} alpha_{m,k}.
bool lssp_coefficients(int m, double* out)
{
    typedef __int128 i128;
    struct Q { i128 p, q; };
    auto gcd = [](i128 a, i128 b) {
        if (a < 0) a = -a;
        while (b != 0) { i128 t = a % b; a = b; b = t; }
        return a;
    };
    auto make = [&](i128 p, i128 q) {
        i128 g = gcd(p, q);
        if (g == 0) g = 1;
        return Q{p / g, q / g};
    };
    std::vector<Q> a = {Q{0, 1}, Q{1, 1}};
    for (int mm = 3; mm <= m; ++mm) {
        std::vector<Q> c(mm, Q{0, 1});
        for (int k = 1; k <= mm - 2; ++k) c[k] = make(2 * a[k - 1].p, k * a[k - 1].q);
        c[mm - 1] = make(2 * a[mm - 2].p, mm * a[mm - 2].q);
        Q sum{0, 1};
        for (int k = 1; k < mm; ++k) sum = make(sum.p * c[k].q + c[k].p * sum.q, sum.q * c[k].q);
        c[0] = make(sum.q - sum.p, sum.q);
        a = c;
    }
    const i128 lim = ((i128)1) << 53;
    for (int k = 0; k < m; ++k) {
        i128 p = a[k].p < 0 ? -a[k].p : a[k].p;
        if (p >= lim || a[k].q >= lim) return false;
        out[k] = (double)(long long)a[k].p / (double)(long long)a[k].q;
    }
    return true;
}

enomr_status check_lssp(const enomr_problem* prob, int m)
{
    if (enomr_status st = check_problem(prob)) return st;
    if (prob->ndim != 1 || prob->system == ENOMR_EULER)
        return fail(ENOMR_EINVAL, "linear SSP-RK is provided for scalar 1D problems");
    if (m < 2 || m > kMaxLsspStages) return fail(ENOMR_EINVAL, "m must be in 2..18");
    return ENOMR_OK;
}

// The problem's workspace, then m stage states, L, and device scalars.
size_t lssp_stage_offset(const enomr_problem& p) { return align_up(layout(p).total); }

}  // namespace

enomr_status enomr_lssp_workspace_size(const enomr_problem* prob, int m, size_t* bytes)
{
    if (enomr_status st = check_lssp(prob, m)) return st;
    if (!bytes) return fail(ENOMR_EINVAL, "bytes is NULL");
    const size_t line = align_up(sizeof(double) * (size_t)prob->nx);
    *bytes = lssp_stage_offset(*prob) + (size_t)(m + 1) * line + 256 + align_up(sizeof(double) * kMaxLsspStages);
    return ENOMR_OK;
}

enomr_status enomr_lssp_advance(enomr_ctx* ctx, const enomr_problem* prob, double* U, double dt, int64_t nsteps,
                                int m, void* ws)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_lssp(prob, m)) return st;
    if (!U || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (!(dt > 0.0) || nsteps < 0) return fail(ENOMR_EINVAL, "bad dt or nsteps");
    double coef[kMaxLsspStages];
    if (!lssp_coefficients(m, coef)) return fail(ENOMR_EINVAL, "coefficients not representable");
    const enomr_problem& p = *prob;
    const long n = p.nx;
    const size_t line = align_up(sizeof(double) * (size_t)n);
    char* base = static_cast<char*>(ws) + lssp_stage_offset(p);
    // stage k at base + k * line; then L, hdt and the coefficients
    double* L = reinterpret_cast<double*>(base + (size_t)m * line);
    double* hdt = reinterpret_cast<double*>(base + (size_t)(m + 1) * line);
    double* dcoef = reinterpret_cast<double*>(base + (size_t)(m + 1) * line + 256);
    HIP_TRY(hipMemcpyAsync(dcoef, coef, sizeof(double) * m, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, ctx->stream, hdt, 1L, 0.5 * dt);
    HIP_TRY(hipGetLastError());
    auto stage = [&](int k) { return reinterpret_cast<double*>(base + (size_t)k * line); };
    for (int64_t step = 0; step < nsteps; ++step) {
        HIP_TRY(hipMemcpyAsync(stage(0), U, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream));
        for (int s = 1; s < m; ++s) {
            if (enomr_status st = launch_alpha(ctx, p, stage(s - 1), ws, nullptr)) return st;
            StageOut so;
            so.Un = stage(s - 1);
            so.Lprev = nullptr;
            so.out = stage(s);
            so.dt = hdt;
            so.stage = 1;   // u^(s) = u^(s-1) + hdt L(u^(s-1))
            if (enomr_status st = launch_operator(ctx, p, stage(s - 1), so, nullptr, ws, nullptr)) return st;
        }
        if (enomr_status st = launch_alpha(ctx, p, stage(m - 1), ws, nullptr)) return st;
        StageOut so;
        so.Un = nullptr;
        so.Lprev = nullptr;
        so.out = L;
        so.dt = nullptr;
        so.stage = 0;
        if (enomr_status st = launch_operator(ctx, p, stage(m - 1), so, nullptr, ws, nullptr)) return st;
        hipLaunchKernelGGL(k_lssp_combine, dim3(blocks_for(n, 256)), dim3(256), 0, ctx->stream, stage(0),
                           (long)(line / sizeof(double)), n, m, dcoef, L, hdt, U);
        HIP_TRY(hipGetLastError());
    }
    return ENOMR_OK;
}

enomr_status enomr_profile_start(enomr_ctx* ctx)
{
    if (!ctx) return fail(ENOMR_EINVAL, "context is NULL");
    ctx->prof = true;
    for (auto& u : ctx->used) u = 0;
    return ENOMR_OK;
}

enomr_status enomr_profile_stop(enomr_ctx* ctx, double* ms, int64_t* launches)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    ctx->prof = false;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < PROF_CLASSES; ++c) {
        double tot = 0.0;
        for (size_t i = 0; i < ctx->used[c]; ++i) {
            float e = 0.0f;
            HIP_TRY(hipEventElapsedTime(&e, ctx->ev[c][i].first, ctx->ev[c][i].second));
            tot += e;
        }
        if (ms) ms[c] = tot;
        if (launches) launches[c] = (int64_t)ctx->used[c];
    }
    return ENOMR_OK;
}

enomr_status enomr_check(enomr_ctx* ctx)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    unsigned h = 0;
    HIP_TRY(hipMemcpy(&h, ctx->status, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (h) {
        HIP_TRY(hipMemset(ctx->status, 0, sizeof(unsigned)));
        return fail(ENOMR_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or NaN) met on the device");
    }
    return ENOMR_OK;
}


// ---------------------------------------------------------------------------
// Frozen-stencil adjoint (1D Euler)
// ---------------------------------------------------------------------------

enomr_status enomr_rhs_adjoint(enomr_ctx* ctx, const enomr_problem* prob, const double* U, const uint8_t* idx,
                               const double* alpha_dev, const double* lam_dUdt, double* lam_U, void* ws)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_adjoint_problem(prob)) return st;
    if (!U || !idx || !alpha_dev || !lam_dUdt || !lam_U || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (lam_U == lam_dUdt) return fail(ENOMR_EINVAL, "lam_U must not alias lam_dUdt");
    AdjIn a{};
    a.U = U;
    a.idx = idx;
    a.alpha = alpha_dev;
    a.lamIn = lam_dUdt;
    a.dt = nullptr;
    a.a = 0.0;
    a.b = 1.0;
    a.cb = 0.0;
    a.lamOut = lam_U;
    return launch_adjoint_stage(ctx, *prob, a);
}

enomr_status enomr_record_steps(enomr_ctx* ctx, const enomr_problem* prob, double* U, double cfl, int64_t nsteps,
                                double* stages, uint8_t* idx_log, double* alpha_log, double* dt_log, void* ws)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_adjoint_problem(prob)) return st;
    if (!U || !stages || !idx_log || !alpha_log || !dt_log || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (!(cfl > 0.0) || nsteps < 0) return fail(ENOMR_EINVAL, "bad cfl or nsteps");
    return record_steps(ctx, *prob, U, cfl, nsteps, stages, idx_log, alpha_log, dt_log, ws);
}

enomr_status enomr_adjoint_steps(enomr_ctx* ctx, const enomr_problem* prob, int64_t nsteps, const double* stages,
                                 const uint8_t* idx_log, const double* alpha_log, const double* dt_log, double* lam,
                                 void* ws)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (enomr_status st = check_adjoint_problem(prob)) return st;
    if (!stages || !idx_log || !alpha_log || !dt_log || !lam || !ws) return fail(ENOMR_EINVAL, "NULL array");
    if (nsteps < 0) return fail(ENOMR_EINVAL, "bad nsteps");
    return adjoint_steps(ctx, *prob, nsteps, stages, idx_log, alpha_log, dt_log, lam, ws);
}

// ---------------------------------------------------------------------------
// Batched persistent execution
// ---------------------------------------------------------------------------

namespace {

const int kBatchTF[3] = {64, 128, 256};

hipError_t launch_batch(enomr_batch* b, int tf, const BatchProb* probs, hipStream_t st)
{
    switch (tf) {
    case 64:
        hipLaunchKernelGGL(k_batch_euler1d<64>, dim3(b->nblocks), dim3(64), 0, st, probs, b->d_order, b->nprob,
                           b->d_queue, b->d_params, b->ctx->status);
        break;
    case 128:
        hipLaunchKernelGGL(k_batch_euler1d<128>, dim3(b->nblocks), dim3(128), 0, st, probs, b->d_order, b->nprob,
                           b->d_queue, b->d_params, b->ctx->status);
        break;
    default:
        hipLaunchKernelGGL(k_batch_euler1d<256>, dim3(b->nblocks), dim3(256), 0, st, probs, b->d_order, b->nprob,
                           b->d_queue, b->d_params, b->ctx->status);
        break;
    }
    return hipGetLastError();
}

// Tile shapes of the batched 2D kernel (faces per line, lines).
constexpr int kB2Shapes[3][2] = {{64, 4}, {32, 8}, {16, 16}};

#define DISPATCH_SHAPE2(shape, ...)                                             \
    switch (shape) {                                                            \
    case 0: { constexpr int TF = 64, TL = 4; __VA_ARGS__; } break;              \
    case 2: { constexpr int TF = 16, TL = 16; __VA_ARGS__; } break;             \
    default: { constexpr int TF = 32, TL = 8; __VA_ARGS__; } break;             \
    }

// One SSP-RK3 step of one order's 2D problems on stream st: per stage the
// alphas (and at the first stage dt), the y sweep, the x sweep.
hipError_t launch_b2_group(const enomr_batch* b, int shape, const enomr_batch::Group2& g, const BatchProb2* probs,
                           hipStream_t st)
{
    const int2* tx = b->d_tiles2 + g.off[shape][0];
    const int2* ty = b->d_tiles2 + g.off[shape][1];
    const unsigned nx = (unsigned)g.tiles[shape][0], ny = (unsigned)g.tiles[shape][1];
    unsigned* status = b->ctx->status;
    for (int stage = 1; stage <= 3; ++stage) {
        hipLaunchKernelGGL(k_batch2_alpha, dim3(g.count), dim3(kB2AlphaNT), 0, st, probs, b->d_list2 + g.first, stage,
                           b->d_params, status);
        DISPATCH_SHAPE2(shape, DISPATCH_R(2 * g.R - 1,
            hipLaunchKernelGGL((k_batch2_sweep<R, 1, TF, TL>), dim3(ny), dim3(TF * TL), 0, st, probs, ty, stage, status);
            hipLaunchKernelGGL((k_batch2_sweep<R, 0, TF, TL>), dim3(nx), dim3(TF * TL), 0, st, probs, tx, stage, status)));
    }
    return hipGetLastError();
}

long b2_tiles(int shape, int dir, long nx, long ny)
{
    long t = 0;
    DISPATCH_SHAPE2(shape, t = dir == 0 ? batch2_tiles<0, TF, TL>(nx, ny) : batch2_tiles<1, TF, TL>(nx, ny));
    return t;
}

unsigned batch_blocks(int tf, int nprob)
{
    int per_cu = 0, ncu = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = hipErrorInvalidValue;
    if (tf == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_euler1d<64>, 64, 0);
    else if (tf == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_euler1d<128>, 128, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_euler1d<256>, 256, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    if (ncu < 1) ncu = 1;
    long nb = (long)per_cu * ncu;
    if (nb > nprob) nb = nprob;
    return (unsigned)(nb < 1 ? 1 : nb);
}

void batch_free(enomr_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->exec2) (void)hipGraphExecDestroy(b->exec2);
    if (b->graph2) (void)hipGraphDestroy(b->graph2);
    if (b->cap2) (void)hipStreamDestroy(b->cap2);
    for (hipStream_t st : b->br) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : b->brev) (void)hipEventDestroy(ev);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->fork2) (void)hipEventDestroy(b->fork2);
    (void)hipFree(b->d_probs);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_probs2);
    (void)hipFree(b->d_list2);
    (void)hipFree(b->d_tiles2);
    (void)hipFree(b->d_queue);
    (void)hipFree(b->d_params);
    (void)hipFree(b->d_ws);
    delete b;
}

}  // namespace

// Capture the 1D problems' persistent launch into a graph (all steps), and
// one step of the 2D problems into another, one branch per order (streams of
// default priority); advance replays the first once and the second once per
// step.  Each replaces the previous one.
enomr_status capture_batch(enomr_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    if (b->nprob == 0) return ENOMR_OK;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(ENOMR_EHIP, "cannot begin capture");
    const hipError_t le = launch_batch(b, b->tf, b->d_probs, b->cap);
    const hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess || ce != hipSuccess) return fail(ENOMR_EHIP, "capture of the batch launch failed");
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(ENOMR_EHIP, "cannot instantiate the batch graph");
    return ENOMR_OK;
}

enomr_status capture_batch2(enomr_batch* b)
{
    if (b->exec2) (void)hipGraphExecDestroy(b->exec2);
    if (b->graph2) (void)hipGraphDestroy(b->graph2);
    b->exec2 = nullptr;
    b->graph2 = nullptr;
    if (b->nprob2 == 0) return ENOMR_OK;
    b->nblocks2 = 0;
    for (const auto& g : b->groups2)
        for (int d = 0; d < 2; ++d) b->nblocks2 = std::max(b->nblocks2, (unsigned)g.tiles[b->shape2][d]);
    if (hipStreamBeginCapture(b->cap2, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(ENOMR_EHIP, "cannot begin capture");
    hipError_t le = hipEventRecord(b->fork2, b->cap2);
    for (size_t k = 0; k < b->groups2.size() && le == hipSuccess; ++k) {
        le = hipStreamWaitEvent(b->br[k], b->fork2, 0);
        if (le == hipSuccess) le = launch_b2_group(b, b->shape2, b->groups2[k], b->d_probs2, b->br[k]);
        if (le == hipSuccess) le = hipEventRecord(b->brev[k], b->br[k]);
        if (le == hipSuccess) le = hipStreamWaitEvent(b->cap2, b->brev[k], 0);
    }
    const hipError_t ce = hipStreamEndCapture(b->cap2, &b->graph2);
    if (le != hipSuccess || ce != hipSuccess) return fail(ENOMR_EHIP, "capture of the 2D batch step failed");
    if (hipGraphInstantiate(&b->exec2, b->graph2, nullptr, nullptr, 0) != hipSuccess)
        return fail(ENOMR_EHIP, "cannot instantiate the 2D batch graph");
    return ENOMR_OK;
}

enomr_status enomr_batch_create(enomr_ctx* ctx, int32_t nprob, const enomr_problem* probs, double* const* U,
                                int autotune, enomr_batch** out)
{
    if (enomr_status st = check_ctx(ctx)) return st;
    if (!out || !probs || !U || nprob < 1) return fail(ENOMR_EINVAL, "bad batch arguments");
    if (autotune != 0 && autotune != 1 && autotune != 64 && autotune != 128 && autotune != 256)
        return fail(ENOMR_EINVAL, "autotune must be 0, 1, 64, 128 or 256");
    *out = nullptr;
    // 1D problems (index list i1) and 2D problems (i2), each with its stage workspace
    std::vector<int> i1, i2;
    size_t total = 0;
    for (int i = 0; i < nprob; ++i) {
        const enomr_problem& p = probs[i];
        if (enomr_status st = check_problem(&p)) return st;
        if (p.system != ENOMR_EULER) return fail(ENOMR_EINVAL, "batched problems must be Euler problems");
        if (!default_operator(p)) return fail(ENOMR_EINVAL, "batched problems take the default operator only");
        if (!U[i]) return fail(ENOMR_EINVAL, "NULL state in batch");
        if (p.ndim == 1) {
            i1.push_back(i);
            total += align_up(sizeof(double) * 3 * (size_t)p.nx) * 2;
        } else {
            i2.push_back(i);
            const size_t plane = sizeof(double) * (size_t)p.nx * (size_t)p.ny;
            total += align_up(4 * plane) * 3 + align_up(sizeof(double) * (size_t)p.ny) +
                     align_up(sizeof(double) * (size_t)p.nx) + align_up(sizeof(double));
        }
    }
    enomr_batch* b = new enomr_batch;
    b->ctx = ctx;
    b->nprob = (int)i1.size();
    b->nprob2 = (int)i2.size();
    auto bail = [&](enomr_status st, const std::string& m) {
        batch_free(b);
        return fail(st, m);
    };
    if (hipMalloc(&b->d_ws, total) != hipSuccess) return bail(ENOMR_ENOMEM, "cannot allocate batch workspace");
    char* wsb = reinterpret_cast<char*>(b->d_ws);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        double* p = reinterpret_cast<double*>(wsb + off);
        off += align_up(bytes);
        return p;
    };
    std::vector<BatchProb> hp(b->nprob);
    std::vector<double> cost(b->nprob);
    for (int k = 0; k < b->nprob; ++k) {
        const enomr_problem& p = probs[i1[k]];
        BatchProb& q = hp[k];
        q.U = U[i1[k]];
        q.U1 = take(sizeof(double) * 3 * (size_t)p.nx);
        q.U2 = take(sizeof(double) * 3 * (size_t)p.nx);
        q.n = p.nx;
        q.ih = 1.0 / p.hx;
        q.gamma = p.gamma;
        q.R = (p.order + 1) / 2;
        q.bc = p.bc_x;
        cost[k] = (double)p.nx * (double)(q.R + 3);
    }
    std::vector<BatchProb2> hp2(b->nprob2);
    std::vector<double> cost2(b->nprob2);
    for (int k = 0; k < b->nprob2; ++k) {
        const enomr_problem& p = probs[i2[k]];
        const size_t plane = sizeof(double) * (size_t)p.nx * (size_t)p.ny;
        BatchProb2& q = hp2[k];
        q.U = U[i2[k]];
        q.U1 = take(4 * plane);
        q.U2 = take(4 * plane);
        q.L = take(4 * plane);
        q.ax = take(sizeof(double) * (size_t)p.ny);
        q.ay = take(sizeof(double) * (size_t)p.nx);
        q.dt = take(sizeof(double));
        q.nx = p.nx;
        q.ny = p.ny;
        q.ihx = 1.0 / p.hx;
        q.ihy = 1.0 / p.hy;
        q.gamma = p.gamma;
        q.R = (p.order + 1) / 2;
        q.bcx = p.bc_x;
        q.bcy = p.bc_y;
        cost2[k] = 2.0 * (double)p.nx * (double)p.ny * (double)(q.R + 3);
    }
    // longest first: the work queues then hand out problems in LPT order
    auto lpt = [](const std::vector<double>& c) {
        std::vector<int> o(c.size());
        for (size_t i = 0; i < c.size(); ++i) o[i] = (int)i;
        std::stable_sort(o.begin(), o.end(), [&](int a, int d) { return c[a] > c[d]; });
        return o;
    };
    const std::vector<int> order = lpt(cost), order2 = lpt(cost2);
    // 2D problems by order (ascending), longest first within an order; the
    // tile lists of each order, shape and direction follow its problems
    std::vector<int> list2;
    std::vector<int2> tiles2;
    for (int R = 3; R <= 9; ++R) {
        enomr_batch::Group2 g;
        g.R = R;
        g.first = (int)list2.size();
        for (int k : order2)
            if (hp2[k].R == R) list2.push_back(k);
        g.count = (int)list2.size() - g.first;
        if (g.count == 0) continue;
        b->groups2.push_back(g);
    }
    for (int t = 0; t < 3; ++t)
        for (auto& g : b->groups2)
            for (int d = 0; d < 2; ++d) {
                g.off[t][d] = (long)tiles2.size();
                for (int i = g.first; i < g.first + g.count; ++i) {
                    const long nt = b2_tiles(t, d, hp2[list2[i]].nx, hp2[list2[i]].ny);
                    for (long j = 0; j < nt; ++j) tiles2.push_back(make_int2(list2[i], (int)j));
                }
                g.tiles[t][d] = (long)tiles2.size() - g.off[t][d];
            }
    if (hipMalloc(&b->d_queue, sizeof(int) * 2) != hipSuccess || hipMalloc(&b->d_params, sizeof(BatchParams)) != hipSuccess)
        return bail(ENOMR_ENOMEM, "cannot allocate batch descriptors");
    if (b->nprob > 0) {
        if (hipMalloc(&b->d_probs, sizeof(BatchProb) * b->nprob) != hipSuccess ||
            hipMalloc(&b->d_order, sizeof(int) * b->nprob) != hipSuccess)
            return bail(ENOMR_ENOMEM, "cannot allocate batch descriptors");
        if (hipMemcpy(b->d_probs, hp.data(), sizeof(BatchProb) * b->nprob, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->d_order, order.data(), sizeof(int) * b->nprob, hipMemcpyHostToDevice) != hipSuccess)
            return bail(ENOMR_EHIP, "cannot upload batch descriptors");
    }
    if (b->nprob2 > 0) {
        if (hipMalloc(&b->d_probs2, sizeof(BatchProb2) * b->nprob2) != hipSuccess ||
            hipMalloc(&b->d_list2, sizeof(int) * list2.size()) != hipSuccess ||
            hipMalloc(&b->d_tiles2, sizeof(int2) * tiles2.size()) != hipSuccess)
            return bail(ENOMR_ENOMEM, "cannot allocate batch descriptors");
        if (hipMemcpy(b->d_probs2, hp2.data(), sizeof(BatchProb2) * b->nprob2, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->d_list2, list2.data(), sizeof(int) * list2.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->d_tiles2, tiles2.data(), sizeof(int2) * tiles2.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(ENOMR_EHIP, "cannot upload batch descriptors");
    }

    // Autotune the 1D kernel's tile width: one step of the 1D problems on
    // scratch copies of their states, per width; the fastest wins.
    b->tf = 128;
    if (autotune == 64 || autotune == 128 || autotune == 256) b->tf = autotune;
    const int n1 = b->nprob;
    if (autotune == 1 && n1 > 0) {
        size_t state_bytes = 0;
        for (int k = 0; k < n1; ++k) state_bytes += align_up(sizeof(double) * 3 * (size_t)probs[i1[k]].nx);
        double* scratch = nullptr;
        BatchProb* d_tune = nullptr;
        if (hipMalloc(&scratch, state_bytes) != hipSuccess || hipMalloc(&d_tune, sizeof(BatchProb) * n1) != hipSuccess) {
            (void)hipFree(scratch);
            return bail(ENOMR_ENOMEM, "cannot allocate autotune scratch");
        }
        std::vector<BatchProb> tp = hp;
        size_t so = 0;
        for (int k = 0; k < n1; ++k) {
            tp[k].U = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) + so);
            so += align_up(sizeof(double) * 3 * (size_t)probs[i1[k]].nx);
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool ok = hipMemcpy(d_tune, tp.data(), sizeof(BatchProb) * n1, hipMemcpyHostToDevice) == hipSuccess &&
                  hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        double best = 1e300;
        for (int t = 0; ok && t < 3; ++t) {
            const int tf = kBatchTF[t];
            for (int k = 0; k < n1 && ok; ++k)
                ok = hipMemcpyAsync(tp[k].U, U[i1[k]], sizeof(double) * 3 * (size_t)probs[i1[k]].nx,
                                    hipMemcpyDeviceToDevice, ctx->stream) == hipSuccess;
            b->nblocks = batch_blocks(tf, n1);
            hipLaunchKernelGGL(k_set_batch_params, dim3(1), dim3(64), 0, ctx->stream, b->d_params, 0.5, 1L, b->d_queue);
            ok = ok && hipEventRecord(e0, ctx->stream) == hipSuccess;
            ok = ok && launch_batch(b, tf, d_tune, ctx->stream) == hipSuccess;
            ok = ok && hipEventRecord(e1, ctx->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            b->tune_ms[t] = ms;
            if (ok && ms < best) {
                best = ms;
                b->tf = tf;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(d_tune);
        (void)hipFree(scratch);
        if (!ok) return bail(ENOMR_EHIP, "autotune failed");
        // the autotune steps may have latched a status; keep it for enomr_check
    }
    if (n1 > 0) b->nblocks = batch_blocks(b->tf, n1);

    // Autotune the 2D sweeps' tile shape the same way: one step of the 2D
    // problems on scratch copies of their states, per shape (the orders one
    // after another on the context's stream).
    const int n2 = b->nprob2;
    b->shape2 = 1;
    if (autotune == 1 && n2 > 0) {
        size_t state_bytes = 0;
        for (int k = 0; k < n2; ++k)
            state_bytes += align_up(sizeof(double) * 4 * (size_t)probs[i2[k]].nx * (size_t)probs[i2[k]].ny);
        double* scratch = nullptr;
        BatchProb2* d_tune = nullptr;
        if (hipMalloc(&scratch, state_bytes) != hipSuccess || hipMalloc(&d_tune, sizeof(BatchProb2) * n2) != hipSuccess) {
            (void)hipFree(scratch);
            return bail(ENOMR_ENOMEM, "cannot allocate autotune scratch");
        }
        std::vector<BatchProb2> tp = hp2;
        size_t so = 0;
        for (int k = 0; k < n2; ++k) {
            tp[k].U = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) + so);
            so += align_up(sizeof(double) * 4 * (size_t)probs[i2[k]].nx * (size_t)probs[i2[k]].ny);
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool ok = hipMemcpy(d_tune, tp.data(), sizeof(BatchProb2) * n2, hipMemcpyHostToDevice) == hipSuccess &&
                  hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        double best = 1e300;
        for (int t = 0; ok && t < 3; ++t) {
            for (int k = 0; k < n2 && ok; ++k)
                ok = hipMemcpyAsync(tp[k].U, U[i2[k]],
                                    sizeof(double) * 4 * (size_t)probs[i2[k]].nx * (size_t)probs[i2[k]].ny,
                                    hipMemcpyDeviceToDevice, ctx->stream) == hipSuccess;
            hipLaunchKernelGGL(k_set_batch_params, dim3(1), dim3(64), 0, ctx->stream, b->d_params, 0.5, 1L, b->d_queue);
            ok = ok && hipEventRecord(e0, ctx->stream) == hipSuccess;
            for (const auto& g : b->groups2) ok = ok && launch_b2_group(b, t, g, d_tune, ctx->stream) == hipSuccess;
            ok = ok && hipEventRecord(e1, ctx->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            b->tune2_ms[t] = ms;
            if (ok && ms < best) {
                best = ms;
                b->shape2 = t;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(d_tune);
        (void)hipFree(scratch);
        if (!ok) return bail(ENOMR_EHIP, "autotune failed");
    }

    bool sok = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess &&
               hipStreamCreateWithFlags(&b->cap2, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&b->join, hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&b->fork2, hipEventDisableTiming) == hipSuccess;
    for (size_t k = 0; sok && k < b->groups2.size(); ++k) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        sok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (sok) b->br.push_back(st);
        sok = sok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (sok) b->brev.push_back(ev);
    }
    if (!sok) return bail(ENOMR_EHIP, "cannot create capture streams");
    if (enomr_status st = capture_batch(b)) {
        batch_free(b);
        return st;
    }
    if (enomr_status st = capture_batch2(b)) {
        batch_free(b);
        return st;
    }
    *out = b;
    return ENOMR_OK;
}

enomr_status enomr_batch_set_tile2d(enomr_batch* b, int32_t tile_faces, int32_t tile_lines)
{
    if (!b) return fail(ENOMR_EINVAL, "batch is NULL");
    if (enomr_status st = check_ctx(b->ctx)) return st;
    int shape = -1;
    for (int t = 0; t < 3; ++t)
        if (kB2Shapes[t][0] == tile_faces && kB2Shapes[t][1] == tile_lines) shape = t;
    if (shape < 0) return fail(ENOMR_EINVAL, "2D tile shape must be 64x4, 32x8 or 16x16");
    // let replays of the current graph finish before it is replaced
    HIP_TRY(hipStreamSynchronize(b->ctx->stream));
    b->shape2 = shape;
    return capture_batch2(b);
}

enomr_status enomr_batch_advance(enomr_batch* b, double cfl, int64_t nsteps)
{
    if (!b) return fail(ENOMR_EINVAL, "batch is NULL");
    if (enomr_status st = check_ctx(b->ctx)) return st;
    if (!(cfl > 0.0) || nsteps < 0) return fail(ENOMR_EINVAL, "bad cfl or nsteps");
    hipStream_t st = b->ctx->stream;
    hipLaunchKernelGGL(k_set_batch_params, dim3(1), dim3(64), 0, st, b->d_params, cfl, (long)nsteps, b->d_queue);
    HIP_TRY(hipGetLastError());
    // the 1D launch (all steps) runs on its own stream beside the 2D steps
    const bool both = b->exec && b->exec2;
    if (both) {
        HIP_TRY(hipEventRecord(b->fork, st));
        HIP_TRY(hipStreamWaitEvent(b->cap, b->fork, 0));
        HIP_TRY(hipGraphLaunch(b->exec, b->cap));
        HIP_TRY(hipEventRecord(b->join, b->cap));
    } else if (b->exec) {
        HIP_TRY(hipGraphLaunch(b->exec, st));
    }
    if (b->exec2)
        for (int64_t k = 0; k < nsteps; ++k) HIP_TRY(hipGraphLaunch(b->exec2, st));
    if (both) HIP_TRY(hipStreamWaitEvent(st, b->join, 0));
    return ENOMR_OK;
}

enomr_status enomr_batch_info2d(const enomr_batch* b, int32_t* tile_faces, int32_t* tile_lines, double* tune_ms)
{
    if (!b) return fail(ENOMR_EINVAL, "batch is NULL");
    if (tile_faces) *tile_faces = kB2Shapes[b->shape2][0];
    if (tile_lines) *tile_lines = kB2Shapes[b->shape2][1];
    if (tune_ms)
        for (int i = 0; i < 3; ++i) tune_ms[i] = b->tune2_ms[i];
    return ENOMR_OK;
}

enomr_status enomr_batch_info(const enomr_batch* b, int32_t* tile_faces, int32_t* workgroups, double* tune_ms)
{
    if (!b) return fail(ENOMR_EINVAL, "batch is NULL");
    if (tile_faces) *tile_faces = b->tf;
    if (workgroups) *workgroups = (int32_t)(b->nblocks + b->nblocks2);
    if (tune_ms)
        for (int i = 0; i < 3; ++i) tune_ms[i] = b->tune_ms[i];
    return ENOMR_OK;
}

enomr_status enomr_batch_destroy(enomr_batch* b)
{
    if (!b) return ENOMR_OK;
    (void)hipSetDevice(b->ctx->device);
    batch_free(b);
    return ENOMR_OK;
}

}  // extern "C"

#ifdef ENOMR_PHASE_STAMPS
// Instrumented builds only: the phase stamps of the last x-face sweep launch
// (kStampBlocks workgroups x kStampWaves waves x kStampPhases stamps, in that
// order) into `host`, which holds `count` of them.
extern "C" enomr_status enomr_phase_stamps(unsigned long long* host, size_t count)
{
    if (!host || count > (size_t)kStampBlocks * kStampWaves * kStampPhases) return fail(ENOMR_EINVAL, "bad buffer");
    HIP_TRY(hipMemcpyFromSymbol(host, HIP_SYMBOL(enomr::g_phase_stamps), count * sizeof(unsigned long long), 0,
                                hipMemcpyDeviceToHost));
    return ENOMR_OK;
}
#endif
