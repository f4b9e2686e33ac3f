// HIP kernels of the ENO-MR hot path for gfx950 (arXiv 2311.15504).
//
// Data layout: FP64 planes [variable][y][x], x fastest; a 1D problem is one
// row.  A "line" is a row (x-sweep) or a column (y-sweep).  Sweep kernels work
// on tiles of TL lines x TF faces; each tile stages its cells plus r halo
// cells per side in LDS (structure of arrays, so that the lanes of a
// wavefront read consecutive doubles), with boundary conditions applied as an
// index map while loading (periodic wrap or zero-gradient clamp).  A tile
// computes TF faces and the TF-1 cells between them; neighbouring tiles
// overlap by one face.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "eno_device.hpp"

namespace enomr {

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1 };

// Phase stamps of the 2D x-face sweep, in an instrumented build only (compiled
// with ENOMR_PHASE_STAMPS defined; the library's own build has none): lane 0
// of each wave of the first kStampBlocks workgroups records, in its record of
// kStampPhases words,
//   0..8   the shader clock (s_memtime) at every phase boundary of its tile
//          (see sweep_tile); stamp 1 waits for the tile's loads, which the
//          uninstrumented kernel does a little later;
//   9, 10  the real-time clock (s_memrealtime, 100 MHz, one count for the
//          whole device, unlike the shader clock) at the tile's start and
//          after its stores are issued;
//   11     the wave's hardware position: HW_ID (CU, shader engine, SIMD) in
//          the low word, the XCD (XCC_ID) in the high word;
//   12     the real-time clock at the kernel's entry;
//   13     the real-time clock once the tile's stores are acknowledged (the
//          wave waits for them here);
// and enomr_phase_stamps copies the records to the host.
constexpr int kStampBlocks = 20000, kStampWaves = 4, kStampPhases = 14;
#ifdef ENOMR_PHASE_STAMPS
extern __device__ unsigned long long g_phase_stamps[kStampBlocks * kStampWaves * kStampPhases];
__device__ __forceinline__ unsigned long long* stamp_record()
{
    if ((threadIdx.x & 63) != 0 || blockIdx.x >= kStampBlocks || (threadIdx.x >> 6) >= kStampWaves) return nullptr;
    return g_phase_stamps + (blockIdx.x * kStampWaves + (threadIdx.x >> 6)) * kStampPhases;
}
#endif
template <int NV, int DIR>
__device__ __forceinline__ void phase_stamp(int k)
{
#ifdef ENOMR_PHASE_STAMPS
    if constexpr (NV == 4 && DIR == 0) {
        // s_getreg operands: register id | offset << 6 | (bits - 1) << 11
        constexpr int kHwId = 4 | (31 << 11), kXccId = 20 | (3 << 11);
        if (k == 1) __builtin_amdgcn_s_waitcnt(0);
        if (unsigned long long* q = stamp_record()) {
            q[k] = __builtin_amdgcn_s_memtime();
            if (k == 0) {
                q[9] = __builtin_amdgcn_s_memrealtime();
                q[11] = (unsigned long long)(unsigned)__builtin_amdgcn_s_getreg(kHwId) |
                        ((unsigned long long)(unsigned)__builtin_amdgcn_s_getreg(kXccId) << 32);
            }
            if (k == 8) {
                q[10] = __builtin_amdgcn_s_memrealtime();
                __builtin_amdgcn_s_waitcnt(0);
                q[13] = __builtin_amdgcn_s_memrealtime();
            }
        }
    }
#else
    (void)k;
#endif
}
// The kernel's entry (record word 12), instrumented build only.
template <int NV, int DIR>
__device__ __forceinline__ void entry_stamp()
{
#ifdef ENOMR_PHASE_STAMPS
    if constexpr (NV == 4 && DIR == 0) {
        if (unsigned long long* q = stamp_record()) q[12] = __builtin_amdgcn_s_memrealtime();
    }
#endif
}
enum { SYS_ADVECTION = 0, SYS_BURGERS = 1 };

__device__ __forceinline__ long map_cell(long i, long n, int bc)
{
    if (bc == BC_PERIODIC) {
        // callers stay within a few tiles of the line, so one wrap is the
        // rule; the division is only reached on lines shorter than a tile
        long k = i < 0 ? i + n : (i >= n ? i - n : i);
        if (k < 0 || k >= n) {
            k = i % n;
            if (k < 0) k += n;
        }
        return k;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__device__ __forceinline__ void flag_nonphysical(unsigned* status)
{
    atomicOr(status, 1u);
}

// Largest of non-negative doubles through their bit patterns (order preserving).
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v)
{
    atomicMax(reinterpret_cast<unsigned long long*>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// The same reduction with the lane permutation formed at each call (the lane
// index passes an empty asm), for callers inside long loops, where the
// compiler would otherwise hold the six permutation indices through the loop.
__device__ __forceinline__ double wave_max_local(double v)
{
    int lane = (int)__lane_id();
    asm volatile("" : "+v"(lane));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int src = (lane ^ off) << 2;
        const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(v));
        const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(v));
        v = fmax(v, __hiloint2double(hi, lo));
    }
    return v;
}

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------

__global__ void k_fill(double* p, long n, double v)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_set_int(int* p, int v)
{
    if (threadIdx.x == 0) *p = v;
}

// Scalar laws: alpha = max |f'(u)| over the line: |a| for advection (no
// pass over the line), max |u| for Burgers.
__global__ void k_alpha_scalar(const double* __restrict__ u, long n, int flux, double a,
                               double* alpha, const int* active)
{
    if (active && *active == 0) return;
    if (flux == SYS_ADVECTION) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) atomic_max_nonneg(alpha, fabs(a));
        return;
    }
    double m = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        m = fmax(m, fabs(u[i]));
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(alpha, m);
}

// Euler: alpha_x[y] = max_x(|u|+c), alpha_y[x] = max_y(|v|+c) (nv = 4);
// nv = 3: alpha_x[0] = max(|u|+c).  Tile: 64 columns x (4*8) rows per block.
// PF (per-field alphas): three planes per direction, alpha_x[k * ny + y] =
// max_x of |u-c|, |u|, |u+c| for k = 0, 1, 2 (alpha_y likewise with v).
// ax and ay must hold zeros.  The kernel also zeroes zp[0 .. zn-1] (a run's
// other alpha buffer, for the next stage; zn = 0: none), which saves that
// stage a fill launch.
template <int NV, bool PF = false>
__global__ __launch_bounds__(256) void k_alpha_euler(const double* __restrict__ U, long nx, long ny,
                                                      double gamma, double* ax, double* ay,
                                                      unsigned* status, const int* active, double* zp, long zn)
{
    if (active && *active == 0) return;
    {
        const long nth = (long)gridDim.x * gridDim.y * blockDim.x;
        for (long i = ((long)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x; i < zn; i += nth)
            zp[i] = 0.0;
    }
    if constexpr (PF) {
        __shared__ double colf[3][4][64];
        const long plane = nx * ny;
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const long x = blockIdx.x * 64L + tx;
        const long y0 = blockIdx.y * 32L;
        const double gm1 = gamma - 1.0;
        double cm[3] = {0.0, 0.0, 0.0};
        for (int r = ty; r < 32; r += 4) {
            const long y = y0 + r;
            double sx[3] = {0.0, 0.0, 0.0}, sy[3] = {0.0, 0.0, 0.0};
            if ((x < nx) && (y < ny)) {
                const long g = y * nx + x;
                const double rho = U[g], m = U[plane + g];
                const double n = NV == 4 ? U[2 * plane + g] : 0.0;
                const double E = U[(NV - 1) * plane + g];
                const double ir = 1.0 / rho;
                const double u = m * ir;
                const double v = NV == 4 ? n * ir : 0.0;
                const double ke = NV == 4 ? 0.5 * (m * u + n * v) : 0.5 * (m * u);
                const double p = gm1 * (E - ke);
                if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(m) || !isfinite(n))
                    flag_nonphysical(status);
                const double c = sqrt((gamma * p) * ir);
                sx[0] = fabs(u - c); sx[1] = fabs(u); sx[2] = fabs(u + c);
                sy[0] = fabs(v - c); sy[1] = fabs(v); sy[2] = fabs(v + c);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double rmax = wave_max(sx[k]);
                if (tx == 0 && y < ny) atomic_max_nonneg(&ax[k * ny + y], rmax);
                cm[k] = fmax(cm[k], sy[k]);
            }
        }
        if (NV == 4) {
#pragma unroll
            for (int k = 0; k < 3; ++k) colf[k][ty][tx] = cm[k];
            __syncthreads();
            if (ty == 0 && x < nx) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double v = fmax(fmax(colf[k][0][tx], colf[k][1][tx]), fmax(colf[k][2][tx], colf[k][3][tx]));
                    atomic_max_nonneg(&ay[k * nx + x], v);
                }
            }
        }
        return;
    }
    __shared__ double col[4][64];
    const long plane = nx * ny;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const long x = blockIdx.x * 64L + tx;
    const long y0 = blockIdx.y * 32L;
    const double gm1 = gamma - 1.0;
    double cmax = 0.0;
    for (int r = ty; r < 32; r += 4) {
        const long y = y0 + r;
        double sx = 0.0, sy = 0.0;
        const bool ok = (x < nx) && (y < ny);
        if (ok) {
            const long g = y * nx + x;
            const double rho = U[g], m = U[plane + g];
            const double n = NV == 4 ? U[2 * plane + g] : 0.0;
            const double E = U[(NV - 1) * plane + g];
            const double ir = 1.0 / rho;
            const double u = m * ir;
            const double v = NV == 4 ? n * ir : 0.0;
            const double ke = NV == 4 ? 0.5 * (m * u + n * v) : 0.5 * (m * u);
            const double p = gm1 * (E - ke);
            if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(m) || !isfinite(n))
                flag_nonphysical(status);
            const double c = sqrt((gamma * p) * ir);
            sx = fabs(u) + c;
            sy = fabs(v) + c;
        }
        const double rmax = wave_max(sx);
        if (tx == 0 && y < ny) atomic_max_nonneg(&ax[y], rmax);
        cmax = fmax(cmax, sy);
    }
    if (NV == 4) {
        col[ty][tx] = cmax;
        __syncthreads();
        if (ty == 0 && x < nx) {
            const double v = fmax(fmax(col[0][tx], col[1][tx]), fmax(col[2][tx], col[3][tx]));
            atomic_max_nonneg(&ay[x], v);
        }
    }
}

// dt from the CFL rule (one block).  1D: dt = cfl / (ax[0] * ihx);
// 2D: dt = cfl / (max(ax) * ihx + max(ay) * ihy).  With t_end > 0, the step
// is cut to end at t_end and *active turns 0 once t has reached it.
__global__ __launch_bounds__(256) void k_dt(const double* ax, long nax, const double* ay, long nay,
                                            double cfl, double ihx, double ihy, double t_end,
                                            double* dt, double* t, int* active, double* dt_log,
                                            long step)
{
    __shared__ double red[2][4];
    double sx = 0.0, sy = 0.0;
    for (long i = threadIdx.x; i < nax; i += 256) sx = fmax(sx, ax[i]);
    for (long i = threadIdx.x; i < nay; i += 256) sy = fmax(sy, ay[i]);
    sx = wave_max(sx);
    sy = wave_max(sy);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sx;
        red[1][threadIdx.x >> 6] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sx = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
        sy = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        double d = nay > 0 ? cfl / (sx * ihx + sy * ihy) : cfl / (sx * ihx);
        if (t_end > 0.0) {
            if (*active == 0 || *t >= t_end) {
                *active = 0;
                d = 0.0;
            } else {
                if (*t + d > t_end) d = t_end - *t;
                *t = *t + d;
            }
        }
        *dt = d;
        if (dt_log) dt_log[step] = d;
    }
}

// ---------------------------------------------------------------------------
// Bare reconstruction at n faces (Sec. 3.2), window read from global memory.
// ---------------------------------------------------------------------------

template <int R, int S>
__global__ __launch_bounds__(256) void k_recon_faces(const double* __restrict__ f, long n,
                                                     double* __restrict__ fhat, uint8_t* idx)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i >= n) return;
    double w[2 * R - 1];
    const long base = S > 0 ? i : i + 1;
#pragma unroll
    for (int k = 0; k < 2 * R - 1; ++k) w[k] = f[base + k];
    int id;
    fhat[i] = recon<R, S>(w, id);
    if (idx) idx[i] = (uint8_t)id;
}

// ---------------------------------------------------------------------------
// SSP-RK3 stage combination (Sec. 2.3, Eq. TVD3rdRK).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double rk_combine(int stage, double un, double us, double L, double dt)
{
    const double e = us + dt * L;
    if (stage == 1) return e;
    if (stage == 2) return 0.75 * un + 0.25 * e;
    return (1.0 / 3.0) * un + (2.0 / 3.0) * e;
}

struct StageOut {
    const double* Un;      // step-start state (RK mode)
    const double* Lprev;   // operator part to add first (2D: L_y in the x sweep), nullable
    double* out;           // L (store mode) or the next stage state (RK mode)
    const double* dt;      // device dt (RK mode)
    int stage;             // 1..3; 0 = store L
};

// ---------------------------------------------------------------------------
// Scalar conservation law on one line: LF split, f^+ and f^- reconstruction,
// conservative difference, then store L or combine an RK stage.
// ---------------------------------------------------------------------------

template <int R, int TF>
__global__ __launch_bounds__(TF) void k_scalar_sweep(const double* __restrict__ us, long n, double ih,
                                                     int flux, double a, int split, int bc,
                                                     const double* alpha, StageOut so, uint8_t* idx,
                                                     const int* active)
{
    if (active && *active == 0) return;
    constexpr int TC = TF - 1;
    constexpr int NCL = TF + 2 * R - 1;
    __shared__ double sp[NCL], sm[NCL], sf[TF];
    const long c0 = blockIdx.x * (long)TC;
    const double al = split ? *alpha : 0.0;
    // the output cell's operands, requested first so that their latency
    // overlaps the staging and the reconstruction
    const int tf = threadIdx.x;
    const long cell = c0 + tf;
    const bool outc = tf < TC && cell < n;
    const double lp_c = (outc && so.Lprev) ? so.Lprev[cell] : 0.0;
    const double un_c = (outc && so.stage) ? so.Un[cell] : 0.0;
    const double us_c = (outc && so.stage) ? us[cell] : 0.0;
    const double dt_c = so.stage ? *so.dt : 0.0;
    // all of a thread's staging loads first: one memory round trip
    constexpr int NIT = (NCL + TF - 1) / TF;
    double ust[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = threadIdx.x + it * TF;
        if (e < NCL) ust[it] = us[map_cell(c0 - R + e, n, bc)];
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = threadIdx.x + it * TF;
        if (e >= NCL) continue;
        const double u = ust[it];
        const double f = flux == SYS_ADVECTION ? a * u : 0.5 * u * u;
        if (split) {
            const double t = al * u;
            sp[e] = 0.5 * (f + t);
            sm[e] = 0.5 * (f - t);
        } else {
            sp[e] = f;
            sm[e] = 0.0;
        }
    }
    __syncthreads();
    const long face = c0 + tf;
    if (face <= n) {
        const int jp = tf + R - 1;   // left cell of the face in LDS
        // the windows are read from the LDS tile as the reconstruction runs
        int ip, im = 0;
        const double hp = recon_streamed<R, +1>(sp + jp - (R - 1), ip);
        double hm = 0.0;
        if (split) hm = recon_streamed<R, -1>(sm + jp - (R - 2), im);
        sf[tf] = hp + hm;
        if (idx) {
            idx[2 * face] = (uint8_t)ip;
            idx[2 * face + 1] = (uint8_t)im;
        }
    }
    __syncthreads();
    if (outc) {
        double L = -((sf[tf + 1] - sf[tf]) * ih);
        if (so.Lprev) L = lp_c + L;
        if (so.stage == 0) so.out[cell] = L;
        else so.out[cell] = rk_combine(so.stage, un_c, us_c, L, dt_c);
    }
}

// The same sweep with the window shared lane to lane instead of through LDS.
// In the component-wise scalar reconstruction neighbouring faces read the
// same split-flux values.  Each lane loads KC = 4 consecutive cells and keeps
// the split fluxes of every cell its four faces read in registers: its own
// cells, and R to the left and R-1 to the right taken from the neighbouring
// lanes by wavefront shifts (DPP wave_shr:1 / wave_shl:1 move all four values
// of a lane one lane over: two 32-bit moves per double).  A wave covers
// 64 KC = 256 cells and reconstructs the faces whose 2R-cell windows lie
// inside it; waves overlap by one face, so every cell's two faces come from
// the same wave.  Four cells per lane keep four loads in flight per lane
// and share each lane's registers between four windows.  No LDS, no barrier.
// The windows hold the same values as the LDS sweep's, so the results are
// the same bit for bit.  Shifts run with every lane of the wave active
// (before any branch on the data); lanes whose faces fall outside the wave
// compute on values they never store.
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    // CTRL 0x130: wave_shl:1 (lane i takes lane i+1); 0x138: wave_shr:1 (lane i
    // takes lane i-1); the edge lane keeps its own value
    const int slo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const int shi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)shi << 32) | (unsigned)slo);
}
__device__ __forceinline__ double from_right(double v) { return wave_shift<0x130>(v); }
__device__ __forceinline__ double from_left(double v) { return wave_shift<0x138>(v); }

constexpr int kScalarKC = 4;   // cells per lane of the lane-shared scalar sweep

// The values at lane-relative cells k = LO .. HI (k = 0 .. KC-1 are the lane's
// own) from the own values v[0 .. KC-1]: out[k - LO].
template <int LO, int HI>
__device__ __forceinline__ void gather_neighbours(const double (&v)[kScalarKC], double (&out)[HI - LO + 1])
{
    constexpr int KC = kScalarKC;
    double cur[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        cur[k] = v[k];
        if (k >= LO && k <= HI) out[k - LO] = v[k];
    }
    // to the left: lane l-1's cells are k - KC
#pragma unroll
    for (int step = 1; step * KC <= -LO + KC - 1; ++step) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            cur[k] = from_left(cur[k]);
            const int rel = k - step * KC;
            if (rel >= LO && rel <= HI) out[rel - LO] = cur[k];
        }
    }
#pragma unroll
    for (int k = 0; k < KC; ++k) cur[k] = v[k];
    // to the right: lane l+1's cells are k + KC
#pragma unroll
    for (int step = 1; step * KC <= HI; ++step) {
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            cur[k] = from_right(cur[k]);
            const int rel = k + step * KC;
            if (rel >= LO && rel <= HI) out[rel - LO] = cur[k];
        }
    }
}

// Wave tiles start at even cells (RA = R rounded up to even cells of left
// halo, an even number CW of cells written), so that a lane's cells pair up
// into 16-byte aligned loads and stores away from the line's ends.
template <int R>
struct DppTile {
    static constexpr int KC = kScalarKC;
    static constexpr int RA = R + (R & 1);                    // left halo, even
    static constexpr int CW = (64 * KC - RA - R) & ~1;        // cells written per wave
};

template <int R>
__global__ __launch_bounds__(256) void k_scalar_sweep_dpp(const double* __restrict__ us, long n, double ih,
                                                          int flux, double a, int split, int bc,
                                                          const double* alpha, StageOut so, uint8_t* idx,
                                                          const int* active)
{
    if (active && *active == 0) return;
    constexpr int KC = kScalarKC;
    constexpr int W = 2 * R - 1;
    constexpr int RA = DppTile<R>::RA, CW = DppTile<R>::CW;
    static_assert(KC % 2 == 0, "cells pair up into 16-byte accesses");
    const int lane = threadIdx.x & 63;
    const long wave = blockIdx.x * 4L + (threadIdx.x >> 6);
    const long base = wave * CW - RA;         // the wave's first cell (wave-local cell 0), even
    const long c0 = base + KC * lane;         // the lane's first cell
    // paired 16-byte accesses where the arrays allow them; the whole wave
    // inside the line: paired loads, no index map
    const bool aligned = (((uintptr_t)us | (uintptr_t)so.out | (so.stage ? (uintptr_t)so.Un : 0)) & 15) == 0;
    const bool inner = aligned && base >= 0 && base + 64 * KC <= n;
    const double al = split ? *alpha : 0.0;
    const double dt = so.stage ? *so.dt : 0.0;   // requested with the cells, used at the end
    // own cells c0 .. c0+KC-1; the stage's U^n at the same cells
    double u[KC], un[KC];
    if (inner) {
#pragma unroll
        for (int k = 0; k < KC; k += 2) {
            const double2 v = *reinterpret_cast<const double2*>(us + c0 + k);
            u[k] = v.x;
            u[k + 1] = v.y;
        }
        if (so.stage) {
#pragma unroll
            for (int k = 0; k < KC; k += 2) {
                const double2 v = *reinterpret_cast<const double2*>(so.Un + c0 + k);
                un[k] = v.x;
                un[k + 1] = v.y;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < KC; ++k) u[k] = us[map_cell(c0 + k, n, bc)];
#pragma unroll
        for (int k = 0; k < KC; ++k) un[k] = (so.stage && c0 + k >= 0 && c0 + k < n) ? so.Un[c0 + k] : 0.0;
    }
    double gp[KC], gm[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const double f = flux == SYS_ADVECTION ? a * u[k] : 0.5 * u[k] * u[k];
        if (split) {
            const double t = al * u[k];
            gp[k] = 0.5 * (f + t);
            gm[k] = 0.5 * (f - t);
        } else {
            gp[k] = f;
            gm[k] = 0.0;
        }
    }
    // face j of the lane (between lane-relative cells j-1 and j) reads f^+ at
    // cells j-R .. j+R-2 and f^- at cells j-R+1 .. j+R-1
    double P[KC + W - 1], M[KC + W - 1];
    gather_neighbours<-R, KC + R - 3>(gp, P);
    gather_neighbours<-R + 1, KC + R - 2>(gm, M);
    double fh[KC];
    int ip[KC], im[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        double wp[W], wm[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            wp[i] = P[j + i];
            wm[i] = M[j + i];
        }
        const double hp = recon<R, +1>(wp, ip[j]);
        double hm = 0.0;
        im[j] = 0;
        if (split) hm = recon<R, -1>(wm, im[j]);
        fh[j] = hp + hm;
    }
    const double fnext = from_right(fh[0]);   // the next lane's first face
    double res[KC];
    bool ok[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        const int F = KC * lane + j;           // wave-local face index
        const long face = base + F;
        if (F >= RA && F <= RA + CW && face <= n && idx) {
            idx[2 * face] = (uint8_t)ip[j];
            idx[2 * face + 1] = (uint8_t)im[j];
        }
        const long cell = face;               // between faces F and F+1
        ok[j] = F >= RA && F <= RA + CW - 1 && cell < n;
        const double right = j + 1 < KC ? fh[j + 1 < KC ? j + 1 : 0] : fnext;
        double L = -((right - fh[j]) * ih);
        if (ok[j] && so.Lprev) L = so.Lprev[cell] + L;
        res[j] = so.stage == 0 ? L : rk_combine(so.stage, un[j], u[j], L, dt);
    }
#pragma unroll
    for (int j = 0; j < KC; j += 2) {
        if (aligned && ok[j] && ok[j + 1]) {
            *reinterpret_cast<double2*>(so.out + c0 + j) = make_double2(res[j], res[j + 1]);
        } else {
            if (ok[j]) so.out[c0 + j] = res[j];
            if (ok[j + 1]) so.out[c0 + j + 1] = res[j + 1];
        }
    }
}

// Last stage of the linear SSP-RK(m, m-1) step (Sec. 2.3, Eq. lSSPRK):
// u = sum_{k < m-1} a_k u^(k) + a_{m-1} (u^(m-1) + hdt L), the sum taken in
// ascending k from zero, each term a product then an add.
// Stage k starts at stages + k * stride.
__global__ void k_lssp_combine(const double* __restrict__ stages, long stride, long n, int m,
                               const double* __restrict__ coef, const double* __restrict__ L,
                               const double* __restrict__ hdt, double* __restrict__ u)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int k = 0; k < m - 1; ++k) acc = acc + coef[k] * stages[k * stride + i];
    u[i] = acc + coef[m - 1] * (stages[(m - 1) * stride + i] + *hdt * L[i]);
}

// ---------------------------------------------------------------------------
// Euler: Roe-averaged eigenvectors at a face (Sec. 4 preamble) and the
// characteristic sweep.
// ---------------------------------------------------------------------------

// Left/right eigenvectors of the face-normal flux Jacobian at the Roe state.
// Fields (u-c, u, [shear,] u+c).  Rows of L and columns of R are kept as the
// distinct entries of the closed forms.
struct Eig {
    double a0, a1, a3, a4;   // first two entries of the u-c and u+c rows of L
    double C, D;             // last entries shared by those rows: -k v/2, k/2
    double l20, ku, kv, k;   // the u row of L: (1 - k q^2/2, k u, k v, -k)
    double u, v, c, H;       // the Roe state, for R
};

template <int NV>
__device__ __forceinline__ bool roe_eigen(double sL, double unL, double utL, double HL, double sR,
                                          double unR, double utR, double HR, double gm1, Eig& e)
{
    const double id = 1.0 / (sL + sR);
    const double u = (sL * unL + sR * unR) * id;
    const double v = NV == 4 ? (sL * utL + sR * utR) * id : 0.0;
    const double H = (sL * HL + sR * HR) * id;
    const double q2 = NV == 4 ? u * u + v * v : u * u;
    const double c2 = gm1 * (H - 0.5 * q2);
    const double c = sqrt(c2);
    const double k = gm1 / c2;
    const double ic = 1.0 / c;
    const double hq = 0.5 * k * q2;
    const double ku = k * u;
    const double uic = u * ic;
    e.a0 = 0.5 * (hq + uic);
    e.a1 = -0.5 * (ku + ic);
    e.a3 = 0.5 * (hq - uic);
    e.a4 = -0.5 * (ku - ic);
    e.kv = k * v;
    e.C = -0.5 * e.kv;
    e.D = 0.5 * k;
    e.l20 = 1.0 - hq;
    e.ku = ku;
    e.k = k;
    e.u = u;
    e.v = v;
    e.c = c;
    e.H = H;
    return c2 > 0.0;
}

// w = L G for all fields.  Each row's chain runs from the last component to
// the first (the rows u-c and u+c then share their last two terms).
// Structural zeros of L are skipped and unit entries added (same value up to
// the sign of a zero result).
template <int NV>
__device__ __forceinline__ void project(const Eig& e, const double (&G)[NV], double (&w)[NV])
{
    if constexpr (NV == 4) {
        const double t = fma(e.C, G[2], e.D * G[3]);
        w[0] = fma(e.a0, G[0], fma(e.a1, G[1], t));
        w[1] = fma(e.l20, G[0], fma(e.ku, G[1], fma(e.kv, G[2], (-e.k) * G[3])));
        w[2] = fma(-e.v, G[0], G[2]);
        w[3] = fma(e.a3, G[0], fma(e.a4, G[1], t));
    } else {
        const double t = e.D * G[2];
        w[0] = fma(e.a0, G[0], fma(e.a1, G[1], t));
        w[1] = fma(e.l20, G[0], fma(e.ku, G[1], (-e.k) * G[2]));
        w[2] = fma(e.a3, G[0], fma(e.a4, G[1], t));
    }
}

// Field Q of L G, the same chain as project<NV> computes for it.
template <int NV, int Q>
__device__ __forceinline__ double project_row(const Eig& e, const double (&G)[NV])
{
    if constexpr (NV == 4) {
        if constexpr (Q == 0) return fma(e.a0, G[0], fma(e.a1, G[1], fma(e.C, G[2], e.D * G[3])));
        if constexpr (Q == 1) return fma(e.l20, G[0], fma(e.ku, G[1], fma(e.kv, G[2], (-e.k) * G[3])));
        if constexpr (Q == 2) return fma(-e.v, G[0], G[2]);
        return fma(e.a3, G[0], fma(e.a4, G[1], fma(e.C, G[2], e.D * G[3])));
    } else {
        if constexpr (Q == 0) return fma(e.a0, G[0], fma(e.a1, G[1], e.D * G[2]));
        if constexpr (Q == 1) return fma(e.l20, G[0], fma(e.ku, G[1], (-e.k) * G[2]));
        return fma(e.a3, G[0], fma(e.a4, G[1], e.D * G[2]));
    }
}

// F-hat = R w-hat, chains over fields 0..NV-1.
template <int NV>
__device__ __forceinline__ void back_project(const Eig& e, const double (&w)[NV], double (&F)[NV])
{
    // u c and q^2/2 from the Roe state again, with the expressions of
    // roe_eigen (the same values); the state passes an empty asm first so
    // that they are formed here, not held from the projection onwards
    double u = e.u, v = e.v, c = e.c;
    asm volatile("" : "+v"(u), "+v"(v), "+v"(c));
    const double uc = u * c;
    const double q2h = 0.5 * (NV == 4 ? u * u + v * v : u * u);
    const double umc = u - c, upc = u + c;
    const double hm = e.H - uc, hp = e.H + uc;
    if constexpr (NV == 4) {
        F[0] = (w[0] + w[1]) + w[3];
        F[1] = fma(upc, w[3], fma(u, w[1], umc * w[0]));
        F[2] = fma(v, w[3], fma(v, w[1], v * w[0]) + w[2]);
        F[3] = fma(hp, w[3], fma(v, w[2], fma(q2h, w[1], hm * w[0])));
    } else {
        F[0] = (w[0] + w[1]) + w[2];
        F[1] = fma(upc, w[2], fma(u, w[1], umc * w[0]));
        F[2] = fma(hp, w[2], fma(q2h, w[1], hm * w[0]));
    }
}

struct SweepIn {
    const double* Us;      // state the operator is evaluated on
    const double* alpha;   // per-line alpha (LF splitting); per-field: [3][lines]
    unsigned* status;
    uint8_t* idx;          // nullable: this direction's stencil log
    const int* active;     // nullable
    long nx, ny;
    double ih, gamma;
    double grav;           // 2D, the sweep adding the other's L: source g [0, 0, rho, rho v] (0: none)
    int bc;
};

// Operator variants of the Euler sweep (compile-time): the characteristic
// reconstruction with one alpha per line (the scheme's default), the
// component-wise reconstruction of G+- = (F +- alpha U)/2 with no projection,
// and per-field alphas: w+-_k = (l_k.F +- alpha_k l_k.U)/2 with alpha_k the
// line's largest |lambda_k|, lambda = (u-c, u, [u,] u+c); the product by
// alpha_k is rounded first, then the sum and the halving.
enum { VAR_CHAR = 0, VAR_COMPONENT = 1, VAR_FIELD = 2 };

// Which of the three per-field alphas field q of an NV-field system uses.
template <int NV>
__device__ constexpr int field_speed(int q)
{
    return q == 0 ? 0 : (q == NV - 1 ? 2 : 1);
}

// The sign-S characteristic values of the cell at LDS entry lp for every
// field.  A, B: the staged arrays (G+ and G- for VAR_CHAR and VAR_COMPONENT;
// F and U for VAR_FIELD); af: the per-field alphas.
template <int NV, int VAR, int S, int NCELL>
__device__ __forceinline__ void char_values(const Eig& e, const double (&A)[NV][NCELL], const double (&B)[NV][NCELL],
                                            const double (&af)[NV], int lp, double (&w)[NV])
{
    if constexpr (VAR == VAR_COMPONENT) {
#pragma unroll
        for (int q = 0; q < NV; ++q) w[q] = S > 0 ? A[q][lp] : B[q][lp];
    } else if constexpr (VAR == VAR_FIELD) {
        double gf[NV], gu[NV], wf[NV], wu[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            gf[q] = A[q][lp];
            gu[q] = B[q][lp];
        }
        project<NV>(e, gf, wf);
        project<NV>(e, gu, wu);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double t = af[q] * wu[q];
            w[q] = S > 0 ? 0.5 * (wf[q] + t) : 0.5 * (wf[q] - t);
        }
    } else {
        double g[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) g[q] = S > 0 ? A[q][lp] : B[q][lp];
        project<NV>(e, g, w);
    }
}

// Field Q of char_values<NV, VAR, S>, the same arithmetic.
template <int NV, int VAR, int S, int Q, int NCELL>
__device__ __forceinline__ double char_value(const Eig& e, const double (&A)[NV][NCELL], const double (&B)[NV][NCELL],
                                             double aq, int lp)
{
    if constexpr (VAR == VAR_COMPONENT) {
        return S > 0 ? A[Q][lp] : B[Q][lp];
    } else if constexpr (VAR == VAR_FIELD) {
        double gf[NV], gu[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            gf[c] = A[c][lp];
            gu[c] = B[c][lp];
        }
        const double wf = project_row<NV, Q>(e, gf);
        const double t = aq * project_row<NV, Q>(e, gu);
        return S > 0 ? 0.5 * (wf + t) : 0.5 * (wf - t);
    } else {
        double g[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) g[c] = S > 0 ? A[c][lp] : B[c][lp];
        return project_row<NV, Q>(e, g);
    }
}

// Window-aligned a_l rows of the candidates beyond the full stencil, in list
// order, for the f^+ window of each order: c_wrow[R][(c-1)(2R-1) + i]
// multiplies window entry i for candidate c = 1 .. n_cands(R)-4 (zero outside
// the stencil).  The f^- row of a candidate is the same row reversed.
constexpr int kRowsMax = (kPool - 4) * kMaxW;
extern __constant__ double c_wrow[10][kRowsMax];

// LDS of one sweep tile: split fluxes and Roe inputs of NCELL staged cells
// (structure of arrays) and the NFACE face fluxes F[q * NFACE + face].  Until
// the face fluxes are written, the F area holds the order's candidate rows
// (c_wrow), which the fallback reads.
template <int NV, int NCELL, int NFACE>
struct SweepLds {
    double Gp[NV][NCELL];
    double Gm[NV][NCELL];
    double Sq[NCELL], Un[NCELL], H[NCELL];
    double Ut[NV == 4 ? NCELL : 1];
    double F[NV * NFACE > kRowsMax ? NV * NFACE : kRowsMax];
};

// Steps 3.1/3.2 beyond the full stencil for field Q and sign S at one face:
// project the sign's window (ascending cells, LDS entries lp0 + i*STEP),
// build its difference table in place, and evaluate the chosen candidate's
// flux chain on a second projection of the window (bitwise the same values;
// re-projecting is cheaper than holding the window in registers).  rows: the
// order's candidate rows in LDS (f^+ frame; f^- reads each row reversed).
template <int NV, int R, int S, int Q, int STEP, int NCELL, int VAR>
__device__ __forceinline__ double fallback_window(const Eig& e, const double (&A)[NV][NCELL],
                                                  const double (&B)[NV][NCELL], double aq, int lp0,
                                                  const double* rows, int& id)
{
    constexpr int W = 2 * R - 1;
    auto proj = [&](int i) { return char_value<NV, VAR, S, Q, NCELL>(e, A, B, aq, lp0 + i * STEP); };
    double w[W];
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = proj(i);
    const double f0 = w[R - 1], lo = w[R - 2], hi = w[R];
    const int c = first_passing<R, S>(w, baseline_is<R, S>(w));
    if (c >= 0) {
        const double* wa = rows + (c - 1) * W;
        double f = wa[S > 0 ? 0 : W - 1] * proj(0);
#pragma unroll
        for (int i = 1; i < W; ++i) f = fma(wa[S > 0 ? i : W - 1 - i], proj(i), f);
        id = c;
        return f;
    }
    return S > 0 ? minmod3<R>(f0, hi, lo, id) : minmod3<R>(f0, lo, hi, id);
}

// One tile of the characteristic ENO-MR sweep: lines line0 .. line0+TL-1,
// faces c0 .. c0+TF-1 (cells c0 .. c0+TF-2).  DIR 0: lines are rows (x faces);
// DIR 1: lines are columns (y faces), evaluated on the permuted state
// (rho, n, m, E) so that the same x-normal formulas apply.  NCL >= TF+2R-1 is
// the number of cells per line the LDS holds.  VAR selects the operator variant (VAR_CHAR,
// VAR_COMPONENT, VAR_FIELD).  All threads of the block must call it.
template <int NV, int R, int DIR, int TF, int TL, int NCL, int VAR = VAR_CHAR, bool LOOPED = false,
          bool SPEED = false>
__device__ __forceinline__ void sweep_tile(const SweepIn& in, const StageOut& so, long line0, long c0,
                                           SweepLds<NV, NCL * TL, TF * TL>& sm, double* smax = nullptr)
{
    // SPEED (1D Euler): fold the largest |u| + c of the cells this thread
    // stores into *smax, with the expressions of block_max_speed, so that the
    // caller has the next stage's alpha without another pass over the line.
    // LOOPED: the caller runs tiles in a loop.  The thread index then passes
    // an empty asm, so that the indices derived from it are formed per tile
    // rather than hoisted out of the loop and held (spilled) through it.
    int tid = threadIdx.x;
    if constexpr (LOOPED) asm volatile("" : "+v"(tid));
    constexpr int NT = TF * TL;
    constexpr int TC = TF - 1;
    constexpr int NCU = TF + 2 * R - 1;   // cells staged per line
    constexpr int W = 2 * R - 1;
    static_assert(NCU <= NCL, "tile stride too small");
    const long nx = in.nx, ny = in.ny, plane = nx * ny;
    const long nlines = DIR == 0 ? ny : nx;
    const long n = DIR == 0 ? nx : ny;
    const double gamma = in.gamma, gm1 = gamma - 1.0;
    // normal-frame component q -> global variable
    auto gvar = [](int q) { return (DIR == 1 && NV == 4) ? (q == 1 ? 2 : (q == 2 ? 1 : q)) : q; };
    auto lpos = [](int line, int cell) { return DIR == 0 ? line * NCL + cell : cell * TL + line; };
    // face fluxes: lanes of a wave are consecutive in both directions' layouts
    auto fpos = [](int line, int f) { return DIR == 0 ? line * TF + f : f * TL + line; };
    auto gidx = [nx](long line, long cell) { return DIR == 0 ? line * nx + cell : cell * nx + line; };

    // ---- stage the tile: primitives, LF split G = (F +- alpha U)/2, Roe inputs.
    // A thread stages up to NIT cells; all their loads (the cells' line alpha
    // included) are issued before any is used, so the staging costs one
    // memory round trip, not NIT.
    constexpr int NE = NCU * TL;
    constexpr int NIT = (NE + NT - 1) / NT;
    double Ust[NIT][NV], alst[NIT];
    // the candidate rows of the fallback, into the face-flux area (free until
    // the fluxes are written)
    constexpr int NROW = (n_cands(R) - 4) * W;
    constexpr int NRIT = (NROW + NT - 1) / NT;
    // Where the face-flux area has room past the candidate rows, each face's
    // Roe H and c wait there for the back-projection (their own slots, written
    // and read by the same thread before the face fluxes overwrite the area)
    // instead of in registers through the reconstruction.
    constexpr bool STASH = VAR != VAR_COMPONENT && NROW + 2 * NT <= (int)(sizeof(sm.F) / sizeof(double));
    double rowv[NRIT];
    phase_stamp<NV, DIR>(0);   // tile start
    __builtin_amdgcn_s_setprio(2);   // issue this tile's loads ahead of other waves' arithmetic
#pragma unroll
    for (int it = 0; it < NRIT; ++it) {
        const int e = tid + it * NT;
        if (e < NROW) rowv[it] = c_wrow[R][e];
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = tid + it * NT;
        const int line = DIR == 0 ? e / NCU : e % TL;
        const int cell = DIR == 0 ? e % NCU : e / TL;
        const long gl = line0 + line;
        if (e < NE && gl < nlines) {
            const long g = gidx(gl, map_cell(c0 - R + cell, n, in.bc));
#pragma unroll
            for (int q = 0; q < NV; ++q) Ust[it][q] = in.Us[gvar(q) * plane + g];
            if constexpr (VAR != VAR_FIELD) alst[it] = in.alpha[gl];
        }
    }
    __builtin_amdgcn_s_setprio(0);
    phase_stamp<NV, DIR>(1);   // the tile's loads have arrived
#pragma unroll
    for (int it = 0; it < NRIT; ++it) {
        const int e = tid + it * NT;
        if (e < NROW) sm.F[e] = rowv[it];
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int e = tid + it * NT;
        const int line = DIR == 0 ? e / NCU : e % TL;
        const int cell = DIR == 0 ? e % NCU : e / TL;
        const long gl = line0 + line;
        if (!(e < NE && gl < nlines)) continue;
        const double (&Uc)[NV] = Ust[it];
        const double rho = Uc[0], mn = Uc[1], E = Uc[NV - 1];
        const double mt = NV == 4 ? Uc[2] : 0.0;
        const double ir = 1.0 / rho;
        const double un = mn * ir;
        const double ut = NV == 4 ? mt * ir : 0.0;
        const double ke = NV == 4 ? 0.5 * (mn * un + mt * ut) : 0.5 * (mn * un);
        const double p = gm1 * (E - ke);
        if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(mn)) flag_nonphysical(in.status);
        double F[NV];
        F[0] = mn;
        F[1] = mn * un + p;
        if constexpr (NV == 4) F[2] = mt * un;
        F[NV - 1] = (E + p) * un;
        const int lp = lpos(line, cell);
        if constexpr (VAR == VAR_FIELD) {
            // F and U as they are: the split follows the projection
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                sm.Gp[q][lp] = F[q];
                sm.Gm[q][lp] = Uc[q];
            }
        } else {
            const double al = alst[it];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const double t = al * Uc[q];
                sm.Gp[q][lp] = 0.5 * (F[q] + t);
                sm.Gm[q][lp] = 0.5 * (F[q] - t);
            }
        }
        if constexpr (VAR != VAR_COMPONENT) {
            sm.Sq[lp] = sqrt(rho);
            sm.Un[lp] = un;
            if constexpr (NV == 4) sm.Ut[lp] = ut;
            sm.H[lp] = (E + p) * ir;
        }
    }
    phase_stamp<NV, DIR>(2);   // staged
    __syncthreads();
    phase_stamp<NV, DIR>(3);   // the whole tile staged

    // Which face a lane takes.  x faces: a wavefront covers FW consecutive
    // faces of 64/FW neighbouring lines (a block rather than a strip of 64
    // faces, so that fewer of its lanes sit idle while those whose windows
    // straddle a discontinuity walk the candidate list), each group of FW
    // lanes reading and writing one row's consecutive doubles.  y faces:
    // lanes run across the TL lines first, the direction of contiguous memory.
    constexpr int FW = TL >= 4 ? 16 : 64 / TL;   // x faces: faces per wavefront row
    constexpr int LW = 64 / FW;                  // x faces: lines per wavefront
    static_assert(DIR == 1 || (TL % LW == 0 && TF % FW == 0 && NT % 64 == 0), "x-face wavefront shape");
    // thread t -> face and line of the tile (wave t / 64, lane t % 64)
    auto lane_face = [](int t) { return DIR == 0 ? ((t / 64) / (TL / LW)) * FW + (t % 64) % FW : t / TL; };
    auto lane_line = [](int t) { return DIR == 0 ? ((t / 64) % (TL / LW)) * LW + (t % 64) / FW : t % TL; };
    const int tf = lane_face(tid);
    const int tl = lane_line(tid);
    const long gl = line0 + tl;
    const long face = c0 + tf;
    const bool live = gl < nlines && face <= n;

    double Fh[NV];
    if (live) {
        const int jp = tf + R - 1;   // left cell of the face in the tile
        const int pl = lpos(tl, jp), pr = lpos(tl, jp + 1);
        Eig e{};
        if constexpr (VAR != VAR_COMPONENT) {
            const bool ok = roe_eigen<NV>(sm.Sq[pl], sm.Un[pl], NV == 4 ? sm.Ut[pl] : 0.0, sm.H[pl], sm.Sq[pr],
                                          sm.Un[pr], NV == 4 ? sm.Ut[pr] : 0.0, sm.H[pr], gm1, e);
            if (!ok) flag_nonphysical(in.status);
            if constexpr (STASH) {
                sm.F[NROW + tid] = e.H;
                sm.F[NROW + NT + tid] = e.c;
            }
        }
        double af[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) af[q] = VAR == VAR_FIELD ? in.alpha[field_speed<NV>(q) * nlines + gl] : 0.0;

        // ---- smooth path: stream the window once, accumulating for every
        // field and sign the full-stencil indicator and flux and keeping the
        // five central values for IS0.  With the characteristic operator the
        // chains run over the split-flux components, and their sums are
        // projected once (the projection is linear); only the five centre
        // cells are projected cell by cell.  The other variants accumulate
        // the characteristic values themselves.
        constexpr int P0 = cand_pool(R, 0);
        constexpr bool SUMS = VAR == VAR_CHAR;
        double hp[NV], hm[NV];
        unsigned fail = 0;
        uint64_t idxw = 0;
        // + sign: stream cells j-r+1 .. j+r-1 once, accumulating the full
        // stencil's indicator and flux; the baseline indicator IS0
        // (Eq. Baseline_IS, centre j) is built as the centre cells go by.
        {
            double is[NV], fl[NV], a[NV], b[NV], cc[NV], isl[NV], is0[NV];
#pragma unroll
            for (int o = -R + 1; o <= R - 1; ++o) {
                double w[NV], x[NV];
                const int lp = lpos(tl, jp + o);
                if constexpr (SUMS) {
#pragma unroll
                    for (int q = 0; q < NV; ++q) x[q] = sm.Gp[q][lp];
                    if (o >= -2 && o <= 2) project<NV>(e, x, w);
                } else {
                    char_values<NV, VAR, +1, NCL * TL>(e, sm.Gp, sm.Gm, af, lp, w);
#pragma unroll
                    for (int q = 0; q < NV; ++q) x[q] = w[q];
                }
                const int ci = o + (R - 1);
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    if (o == -R + 1) {
                        is[q] = kCoef.b[P0][ci] * x[q];
                        fl[q] = kCoef.a[P0][ci] * x[q];
                    } else {
                        is[q] = fma(kCoef.b[P0][ci], x[q], is[q]);
                        fl[q] = fma(kCoef.a[P0][ci], x[q], fl[q]);
                    }
                    if (o == -2) a[q] = w[q];
                    if (o == -1) b[q] = w[q];
                    if (o == 0) {
                        const double f0 = w[q], fm1 = b[q], fm2 = a[q];
                        cc[q] = f0;
                        isl[q] = fmax(fabs(f0 - fm1), fabs(fma(-2.0, fm1, f0) + fm2));
                    }
                    if (o == 1) a[q] = w[q];
                    if (o == 2) {
                        const double f0 = cc[q], fp1 = a[q], fp2 = w[q];
                        is0[q] = fmin(isl[q], fmax(fabs(f0 - fp1), fabs(fma(-2.0, fp1, f0) + fp2)));
                    }
                }
                // Keep both chains advancing cell by cell: without this the
                // compiler sinks them past the loop and holds every projected
                // value in registers.
#pragma unroll
                for (int q = 0; q < NV; ++q) asm volatile("" : "+v"(is[q]), "+v"(fl[q]));
            }
            if constexpr (SUMS) {
                double ps[NV], pf[NV];
                project<NV>(e, is, ps);
                project<NV>(e, fl, pf);
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    is[q] = ps[q];
                    fl[q] = pf[q];
                }
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                hp[q] = fl[q];
                if (is0[q] == 0.0) {
                    // a flat side: no IS can be below 0, minmod gives the centre value
                    hp[q] = cc[q] + 0.5 * 0.0;
                    idxw |= (uint64_t)(n_cands(R) - 1) << (8 * (2 * q));
                } else if (!(fabs(is[q]) < is0[q])) {
                    fail |= 1u << (2 * q);
                }
            }
        }
        // - sign: the mirror image, cells j-r+2 .. j+r, centre j+1 (its upwind
        // side is j+2, j+3; its downwind side j, j-1).
        {
            double is[NV], fl[NV], a[NV], b[NV], cc[NV], isr[NV], is0[NV];
#pragma unroll
            for (int o = -R + 2; o <= R; ++o) {
                double w[NV], x[NV];
                const int lp = lpos(tl, jp + o);
                if constexpr (SUMS) {
#pragma unroll
                    for (int q = 0; q < NV; ++q) x[q] = sm.Gm[q][lp];
                    if (o >= -1 && o <= 3) project<NV>(e, x, w);
                } else {
                    char_values<NV, VAR, -1, NCL * TL>(e, sm.Gp, sm.Gm, af, lp, w);
#pragma unroll
                    for (int q = 0; q < NV; ++q) x[q] = w[q];
                }
                const int ci = R - o;
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    if (o == -R + 2) {
                        is[q] = kCoef.b[P0][ci] * x[q];
                        fl[q] = kCoef.a[P0][ci] * x[q];
                    } else {
                        is[q] = fma(kCoef.b[P0][ci], x[q], is[q]);
                        fl[q] = fma(kCoef.a[P0][ci], x[q], fl[q]);
                    }
                    if (o == -1) a[q] = w[q];
                    if (o == 0) b[q] = w[q];
                    if (o == 1) {
                        const double f0 = w[q], fp1 = b[q], fp2 = a[q];
                        cc[q] = f0;
                        isr[q] = fmax(fabs(f0 - fp1), fabs(fma(-2.0, fp1, f0) + fp2));
                    }
                    if (o == 2) a[q] = w[q];
                    if (o == 3) {
                        const double f0 = cc[q], fm1 = a[q], fm2 = w[q];
                        is0[q] = fmin(fmax(fabs(f0 - fm1), fabs(fma(-2.0, fm1, f0) + fm2)), isr[q]);
                    }
                }
                // Keep both chains advancing cell by cell: without this the
                // compiler sinks them past the loop and holds every projected
                // value in registers.
#pragma unroll
                for (int q = 0; q < NV; ++q) asm volatile("" : "+v"(is[q]), "+v"(fl[q]));
            }
            if constexpr (SUMS) {
                double ps[NV], pf[NV];
                project<NV>(e, is, ps);
                project<NV>(e, fl, pf);
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    is[q] = ps[q];
                    fl[q] = pf[q];
                }
            }
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                hm[q] = fl[q];
                if (is0[q] == 0.0) {
                    hm[q] = cc[q] + 0.5 * 0.0;
                    idxw |= (uint64_t)(n_cands(R) - 1) << (8 * (2 * q + 1));
                } else if (!(fabs(is[q]) < is0[q])) {
                    fail |= 1u << (2 * q + 1);
                }
            }
        }

        constexpr int LSTEP = DIR == 0 ? 1 : TL;   // LDS step between neighbouring cells of a line
        // ---- remaining candidates for the (field, sign) pairs that failed;
        // the pair index is uniform across the wave, so each pass runs code
        // specialised to its field and sign
        phase_stamp<NV, DIR>(4);   // eigenvectors and the full stencil of every pair done
        if (fail) {
#pragma unroll 1
            for (int kk = 0; kk < 2 * NV; ++kk) {
                if (!((fail >> kk) & 1u)) continue;
                int id = 0;
                double res;
                const int lpp = lpos(tl, jp - (R - 1)), lpm = lpos(tl, jp - (R - 2));
                constexpr int NC = NCL * TL;
                switch (kk) {
                case 0: res = fallback_window<NV, R, +1, 0, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[0], lpp, sm.F, id); hp[0] = res; break;
                case 1: res = fallback_window<NV, R, -1, 0, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[0], lpm, sm.F, id); hm[0] = res; break;
                case 2: res = fallback_window<NV, R, +1, 1, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[1], lpp, sm.F, id); hp[1] = res; break;
                case 3: res = fallback_window<NV, R, -1, 1, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[1], lpm, sm.F, id); hm[1] = res; break;
                case 4: res = fallback_window<NV, R, +1, 2, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[2], lpp, sm.F, id); hp[2] = res; break;
                case 5: res = fallback_window<NV, R, -1, 2, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[2], lpm, sm.F, id); hm[2] = res; break;
                case 6:
                    if constexpr (NV == 4) {
                        res = fallback_window<NV, R, +1, 3, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[NV - 1], lpp, sm.F, id);
                        hp[NV - 1] = res;
                    }
                    break;
                default:
                    if constexpr (NV == 4) {
                        res = fallback_window<NV, R, -1, 3, LSTEP, NC, VAR>(e, sm.Gp, sm.Gm, af[NV - 1], lpm, sm.F, id);
                        hm[NV - 1] = res;
                    }
                    break;
                }
                idxw |= (uint64_t)(uint8_t)id << (8 * kk);
            }
        }

        phase_stamp<NV, DIR>(5);   // fallback done
        double wh[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) wh[q] = hp[q] + hm[q];
        if constexpr (VAR == VAR_COMPONENT) {
#pragma unroll
            for (int q = 0; q < NV; ++q) Fh[q] = wh[q];
        } else {
            if constexpr (STASH) {
                e.H = sm.F[NROW + tid];
                e.c = sm.F[NROW + NT + tid];
            }
            back_project<NV>(e, wh, Fh);
        }

        if (in.idx) {
            // the face's line and position from the thread index again
            // (through an empty asm), not held through the reconstruction
            int t = tid;
            asm volatile("" : "+v"(t));
            const long il = line0 + lane_line(t), ifc = c0 + lane_face(t);
            uint8_t* dst = DIR == 0 ? in.idx + ((il * (n + 1) + ifc) * NV) * 2
                                    : in.idx + ((ifc * nx + il) * NV) * 2;
#pragma unroll
            for (int b = 0; b < 2 * NV; ++b) dst[b] = (uint8_t)(idxw >> (8 * b));
        }
    }
    // ---- conservative difference and output; the cell's operands are
    // requested before the barriers so that their latency overlaps them
    // (the cell's position from the thread index again, through an empty
    // asm, rather than held through the reconstruction)
    int ot = tid;
    asm volatile("" : "+v"(ot));
    const int otf = lane_face(ot), otl = lane_line(ot);
    const long ogl = line0 + otl;
    const long cell = c0 + otf;
    const bool outc = ogl < nlines && otf < TC && cell < n;
    const long g = outc ? gidx(ogl, cell) : 0;
    double lp[NV], un[NV], us[NV];
    // the source, added by the 2D sweep that completes the operator: rho and
    // rho v of the cell
    constexpr bool SRC = NV == 4;
    double s_rho = 0.0, s_rv = 0.0;
    double dt = 0.0;
    if (outc) {
        if (so.stage) dt = *so.dt;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const long i = gvar(q) * plane + g;
            lp[q] = so.Lprev ? so.Lprev[i] : 0.0;
            un[q] = so.stage ? so.Un[i] : 0.0;
            us[q] = so.stage ? in.Us[i] : 0.0;
        }
        if (SRC && in.grav != 0.0) {
            s_rho = in.Us[g];
            s_rv = in.Us[2 * plane + g];
        }
    }
    phase_stamp<NV, DIR>(6);   // face flux and the output operands requested
    __syncthreads();   // every fallback is done with the candidate rows
    if (live) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sm.F[q * NT + fpos(tl, tf)] = Fh[q];
    }
    phase_stamp<NV, DIR>(7);   // face fluxes written
    __syncthreads();
    if (outc) {
        double ov[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const int v = gvar(q);
            double L = -((sm.F[q * NT + fpos(otl, otf + 1)] - sm.F[q * NT + fpos(otl, otf)]) * in.ih);
            if (so.Lprev) L = lp[q] + L;
            if (SRC && in.grav != 0.0) {
                if (v == 2) L = L + in.grav * s_rho;
                if (v == 3) L = L + in.grav * s_rv;
            }
            ov[q] = so.stage == 0 ? L : rk_combine(so.stage, un[q], us[q], L, dt);
            so.out[v * plane + g] = ov[q];
        }
        if constexpr (SPEED && NV == 3) {
            const double rho = ov[0], mo = ov[1], E = ov[2];
            const double ir = 1.0 / rho;
            const double u = mo * ir;
            const double ke = 0.5 * (mo * u);
            const double p = gm1 * (E - ke);
            if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(mo)) flag_nonphysical(in.status);
            *smax = fmax(*smax, fabs(u) + sqrt((gamma * p) * ir));
        }
    }
    phase_stamp<NV, DIR>(8);   // output stored
}

// Workgroups are handed to the XCDs round-robin by linear id, and each XCD has
// its own L2.  The linear id is remapped so that every XCD takes runs of
// kXcdRun consecutive tiles, ordered with the tiles that share cache lines
// next to each other: along the line for x faces (shared halo cells), across
// lines for y faces (the lines of neighbouring tiles are neighbouring columns
// of the same rows).  Short runs keep the XCDs' shares of the domain
// interleaved, so the non-smooth regions spread evenly over them.
constexpr unsigned kXcds = 8, kXcdRun = 4;

__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb)
{
    constexpr unsigned G = kXcds * kXcdRun;
    const unsigned g = b / G;
    if ((g + 1) * G > nb) return b;   // last partial group: identity
    const unsigned r = b - g * G;
    return g * G + (r % kXcds) * kXcdRun + r / kXcds;
}

// One tile per workgroup, 1D grid of ceil(n / (TF-1)) x ceil(nlines / TL) tiles.
template <int NV, int R, int DIR, int TF, int TL, int VAR = VAR_CHAR>
__global__ __launch_bounds__(TF* TL, 4) void k_euler_sweep(SweepIn in, StageOut so)
{
    entry_stamp<NV, DIR>();
    if (in.active && *in.active == 0) return;
    constexpr int NCL = TF + 2 * R - 1;
    __shared__ SweepLds<NV, NCL * TL, TF * TL> lds;
    const long n = DIR == 0 ? in.nx : in.ny, nlines = DIR == 0 ? in.ny : in.nx;
    const unsigned nft = (unsigned)((n + TF - 2) / (TF - 1)), nlt = (unsigned)((nlines + TL - 1) / TL);
    const unsigned t = xcd_tile(blockIdx.x, gridDim.x);
    const unsigned ft = DIR == 0 ? t % nft : t / nlt;
    const unsigned lt = DIR == 0 ? t / nft : t % nlt;
    sweep_tile<NV, R, DIR, TF, TL, NCL, VAR>(in, so, (long)lt * TL, (long)ft * (TF - 1), lds);
}

// ---------------------------------------------------------------------------
// Batched persistent execution: many independent 1D Euler problems of uneven
// lengths and orders in one launch.  Each workgroup takes whole problems from
// an atomic queue (host-sorted by decreasing cost) and advances one problem
// through all its steps: per stage a workgroup reduction gives the line's
// alpha (and dt at the first stage), then the line is swept tile by tile with
// the same tile code as the single-problem kernels, so every problem's result
// equals its single-problem run bit for bit.
// ---------------------------------------------------------------------------

struct BatchProb {
    double* U;       // [3][n] state, advanced in place
    double* U1;      // stage states (workspace)
    double* U2;
    long n;
    double ih;
    double gamma;
    int R;           // (order + 1) / 2
    int bc;
};

struct BatchParams {
    double cfl;
    long nsteps;
};

// queue: the work counters of the 1D and the 2D kernel
__global__ void k_set_batch_params(BatchParams* p, double cfl, long nsteps, int* queue)
{
    if (threadIdx.x == 0) {
        p->cfl = cfl;
        p->nsteps = nsteps;
        queue[0] = 0;
        queue[1] = 0;
    }
}

// The largest of the NT threads' values; every thread gets it.
template <int NT>
__device__ __forceinline__ double block_max(double m, double* red)
{
    m = wave_max_local(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

// Largest |u| + c over a 1D Euler line, by every thread of the workgroup (NT
// threads); all threads get the result.
template <int NT>
__device__ __forceinline__ double block_max_speed(const double* __restrict__ U, long n, double gamma,
                                                  unsigned* status, double* red)
{
    const double gm1 = gamma - 1.0;
    double m = 0.0;
    for (long i = threadIdx.x; i < n; i += NT) {
        const double rho = U[i], mo = U[n + i], E = U[2 * n + i];
        const double ir = 1.0 / rho;
        const double u = mo * ir;
        const double ke = 0.5 * (mo * u);
        const double p = gm1 * (E - ke);
        if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(mo)) flag_nonphysical(status);
        m = fmax(m, fabs(u) + sqrt((gamma * p) * ir));
    }
    return block_max<NT>(m, red);
}

// A pointer that every lane holds the same value of, as a scalar.
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p)
{
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}

template <int R, int TF>
__device__ __forceinline__ void run_problem(const BatchProb P, const BatchParams& prm, unsigned* status,
                                            char* lds_raw, double* red, double* s_alpha, double* s_dt)
{
    using Lds = SweepLds<3, TF + 17, TF>;
    Lds& sm = *reinterpret_cast<Lds*>(lds_raw);
    // the state and the two stage buffers as values (a stage picks two of
    // them), not as fields of the descriptor in memory
    double* const u0 = uniform_ptr(P.U);
    double* const u1 = uniform_ptr(P.U1);
    double* const u2 = uniform_ptr(P.U2);
    // the alpha of a stage's input: one pass over the line for the run's
    // first stage, then the stage before folds it into its output phase
    double a_next = 0.0;
    bool known = false;
    for (long step = 0; step < prm.nsteps; ++step) {
        for (int stage = 1; stage <= 3; ++stage) {
            const double* Us = stage == 1 ? u0 : (stage == 2 ? u1 : u2);
            double* out = stage == 1 ? u1 : (stage == 2 ? u2 : u0);
            const double a = known ? a_next : block_max_speed<TF>(Us, P.n, P.gamma, status, red);
            if (threadIdx.x == 0) {
                *s_alpha = a;
                if (stage == 1) *s_dt = prm.cfl / (a * P.ih);
            }
            __syncthreads();
            SweepIn in;
            in.Us = Us;
            in.alpha = s_alpha;
            in.status = status;
            in.idx = nullptr;
            in.active = nullptr;
            in.nx = P.n;
            in.ny = 1;
            in.ih = P.ih;
            in.gamma = P.gamma;
            in.grav = 0.0;
            in.bc = P.bc;
            StageOut so;
            so.Un = u0;
            so.Lprev = nullptr;
            so.out = out;
            so.dt = s_dt;
            so.stage = stage;
            // a tile's staging overwrites the face fluxes the previous tile's
            // output reads
            // each thread's running maximum waits in its own LDS slot, not in
            // a register held through the tile loop
            double smax = 0.0;
            for (long c0 = 0; c0 < P.n; c0 += TF - 1) {
                sweep_tile<3, R, 0, TF, 1, TF + 17, VAR_CHAR, true, true>(in, so, 0, c0, sm, &smax);
                __syncthreads();
            }
            a_next = block_max<TF>(smax, red);
            known = true;
        }
    }
}

template <int TF>
__global__ __launch_bounds__(TF, 4) void k_batch_euler1d(const BatchProb* __restrict__ probs,
                                                         const int* __restrict__ order, int nprob, int* queue,
                                                         const BatchParams* prm, unsigned* status)
{
    __shared__ __align__(16) char lds_raw[sizeof(SweepLds<3, (TF + 17), TF>)];
    __shared__ double red[TF / 64];
    __shared__ double s_alpha, s_dt;
    __shared__ int s_k;
    const BatchParams P = *prm;
    for (;;) {
        if (threadIdx.x == 0) s_k = atomicAdd(queue, 1);
        __syncthreads();
        // the same value in every lane: read as a scalar, so that the
        // problem's descriptor is loaded into scalar registers
        const int k = __builtin_amdgcn_readfirstlane(s_k);
        __syncthreads();
        if (k >= nprob) return;   // the whole workgroup leaves together
        const BatchProb pr = probs[order[k]];
        switch (pr.R) {
        case 3: run_problem<3, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        case 4: run_problem<4, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        case 5: run_problem<5, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        case 6: run_problem<6, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        case 7: run_problem<7, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        case 8: run_problem<8, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        default: run_problem<9, TF>(pr, P, status, lds_raw, red, &s_alpha, &s_dt); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched 2D Euler problems, stage by stage: per stage, one workgroup per
// problem takes its per-line alphas (a wave per row, then per column) and at
// the first stage its dt; then one launch sweeps the y faces of every problem
// of one order and one the x faces (with the RK combination), over a list of
// tiles of all those problems.  The sweeps run the same tile code as the
// single-problem kernels, so every problem's result equals its single-problem
// run bit for bit, and each order has kernels of its own, so that each is
// allocated the registers of its own window.
// ---------------------------------------------------------------------------

struct BatchProb2 {
    double* U;       // [4][ny][nx] state, advanced in place
    double* U1;      // stage states (workspace)
    double* U2;
    double* L;       // L_y (workspace)
    double* ax;      // [ny] alphas of the rows
    double* ay;      // [nx] alphas of the columns
    double* dt;      // the problem's time step (workspace)
    long nx, ny;
    double ihx, ihy;
    double gamma;
    int R;
    int bcx, bcy;
};

// Per-line |u|+c (rows, into ax) and |v|+c (columns, into ay) of one problem
// by the NW waves of a workgroup, the speed formula of k_alpha_euler.  The
// columns go in chunks of 64 (a lane per column, so that every load is a
// row's consecutive doubles); wave w takes rows w, w+NW, ... of a chunk, KR of
// them in flight at once, folding each row's maximum into ax[y] (a row
// belongs to one wave) and keeping its columns' running maxima, which the
// waves then combine through LDS (col: NW x 64 doubles).
template <int NW, int KR>
__device__ __forceinline__ void block_line_speeds_2d(const double* __restrict__ U, long nx, long ny, double gamma,
                                                     unsigned* status, double* ax, double* ay, double* col)
{
    const long plane = nx * ny;
    const double gm1 = gamma - 1.0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (long c0 = 0; c0 < nx; c0 += 64) {
        const long x = c0 + lane;
        const bool xin = x < nx;
        double cm = 0.0;
        for (long y0 = wave; y0 < ny; y0 += (long)NW * KR) {
            double q[KR][4];
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const long y = y0 + (long)k * NW;
                if (xin && y < ny) {
                    const long g = y * nx + x;
#pragma unroll
                    for (int v = 0; v < 4; ++v) q[k][v] = U[v * plane + g];
                }
            }
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const long y = y0 + (long)k * NW;
                if (y >= ny) break;   // uniform across the wave
                double sx = 0.0;
                if (xin) {
                    const double rho = q[k][0], m = q[k][1], nn = q[k][2], E = q[k][3];
                    const double ir = 1.0 / rho;
                    const double u = m * ir;
                    const double v = nn * ir;
                    const double ke = 0.5 * (m * u + nn * v);
                    const double p = gm1 * (E - ke);
                    if (!(rho > 0.0) || !(p > 0.0) || !isfinite(E) || !isfinite(m) || !isfinite(nn))
                        flag_nonphysical(status);
                    const double c = sqrt((gamma * p) * ir);
                    sx = fabs(u) + c;
                    cm = fmax(cm, fabs(v) + c);
                }
                const double r = wave_max(sx);
                if (lane == 0) ax[y] = c0 == 0 ? r : fmax(ax[y], r);
            }
        }
        col[wave * 64 + lane] = cm;
        __syncthreads();
        if (wave == 0 && xin) {
            double m = col[lane];
#pragma unroll
            for (int w = 1; w < NW; ++w) m = fmax(m, col[w * 64 + lane]);
            ay[x] = m;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ const double* batch2_stage_in(const BatchProb2& P, int stage)
{
    return stage == 1 ? P.U : (stage == 2 ? P.U1 : P.U2);
}

// Stage `stage` (1..3) of problems list[0 .. gridDim.x-1], one per workgroup
// of kB2AlphaNT threads: the alphas of the stage input, and at the first stage
// dt = cfl / (max ax / hx + max ay / hy), the expression the single-problem dt
// kernel evaluates.
constexpr int kB2AlphaNT = 512;

__global__ __launch_bounds__(kB2AlphaNT) void k_batch2_alpha(const BatchProb2* __restrict__ probs,
                                                             const int* __restrict__ list, int stage,
                                                             const BatchParams* prm, unsigned* status)
{
    constexpr int NW = kB2AlphaNT / 64;
    __shared__ double col[NW * 64];
    const BatchProb2 P = probs[list[blockIdx.x]];
    const long nx = P.nx, ny = P.ny;
    block_line_speeds_2d<NW, 4>(batch2_stage_in(P, stage), nx, ny, P.gamma, status, P.ax, P.ay, col);
    if (stage != 1) return;   // uniform across the workgroup
    // the lines' alphas were written by other waves: the barrier that ended
    // the last chunk orders them before these reads
    double mx = 0.0, my = 0.0;
    for (long i = threadIdx.x; i < ny; i += blockDim.x) mx = fmax(mx, P.ax[i]);
    for (long i = threadIdx.x; i < nx; i += blockDim.x) my = fmax(my, P.ay[i]);
    mx = wave_max(mx);
    my = wave_max(my);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        col[wave] = mx;
        col[NW + wave] = my;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = col[0];
        my = col[NW];
        for (int w = 1; w < NW; ++w) {
            mx = fmax(mx, col[w]);
            my = fmax(my, col[NW + w]);
        }
        *P.dt = prm->cfl / (mx * P.ihx + my * P.ihy);
    }
}

// One tile per workgroup from tiles[] ({problem, tile}; tile numbered as the
// single-problem sweep numbers its workgroups), all problems of order 2R-1.
// DIR 1: L_y of the stage input into P.L; DIR 0: L_y plus the x part, RK
// stage `stage` combined into the stage output.
template <int R, int TF, int TL>
struct B2Occupancy {
    // workgroups (of four waves) per CU that the LDS allows, at most four
    static constexpr int lds = (int)sizeof(SweepLds<4, (TF + 2 * R - 1) * TL, TF * TL>);
    static constexpr int value = 163840 / lds >= 4 ? 4 : 163840 / lds;
};

template <int R, int DIR, int TF, int TL>
__global__ __launch_bounds__(TF* TL, (B2Occupancy<R, TF, TL>::value)) void k_batch2_sweep(const BatchProb2* __restrict__ probs,
                                                            const int2* __restrict__ tiles, int stage,
                                                            unsigned* status)
{
    constexpr int NCL = TF + 2 * R - 1;
    __shared__ SweepLds<4, NCL * TL, TF * TL> lds;
    const int2 td = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const BatchProb2& P = probs[td.x];
    const long nx = P.nx, ny = P.ny;
    const long n = DIR == 0 ? nx : ny, nlines = DIR == 0 ? ny : nx;
    const unsigned nft = (unsigned)((n + TF - 2) / (TF - 1)), nlt = (unsigned)((nlines + TL - 1) / TL);
    const unsigned t = (unsigned)td.y;
    const unsigned ft = DIR == 0 ? t % nft : t / nlt;
    const unsigned lt = DIR == 0 ? t / nft : t % nlt;
    SweepIn in;
    in.Us = batch2_stage_in(P, stage);
    in.status = status;
    in.idx = nullptr;
    in.active = nullptr;
    in.nx = nx;
    in.ny = ny;
    in.gamma = P.gamma;
    in.grav = 0.0;
    StageOut so;
    if (DIR == 1) {
        in.alpha = P.ay;
        in.ih = P.ihy;
        in.bc = P.bcy;
        so.Un = nullptr;
        so.Lprev = nullptr;
        so.out = P.L;
        so.dt = nullptr;
        so.stage = 0;
    } else {
        in.alpha = P.ax;
        in.ih = P.ihx;
        in.bc = P.bcx;
        so.Un = P.U;
        so.Lprev = P.L;
        so.out = stage == 1 ? P.U1 : (stage == 2 ? P.U2 : P.U);
        so.dt = P.dt;
        so.stage = stage;
    }
    sweep_tile<4, R, DIR, TF, TL, NCL>(in, so, (long)lt * TL, (long)ft * (TF - 1), lds);
}

// The number of tiles of one sweep of an nx x ny problem (the host builds the
// tile lists with it).
template <int DIR, int TF, int TL>
__host__ __device__ constexpr long batch2_tiles(long nx, long ny)
{
    const long n = DIR == 0 ? nx : ny, nlines = DIR == 0 ? ny : nx;
    return ((n + TF - 2) / (TF - 1)) * ((nlines + TL - 1) / TL);
}

}  // namespace enomr
