// flock_kernels.hip -- gfx950 kernels of one flock-environment step.
//
// One step (Sec. 4.1 of arXiv:2207.03945: apply the actions, then update
// view and reward over every pair in spatial proximity; Sec. 2.1: all agents
// update simultaneously) is four dependent phases over a whole batch of
// environments at once.  Agents are kept in cell order between steps (see
// DevEnv), so every phase streams its per-agent data sequentially:
//
//   k_move_count  record p: rotate/accelerate/move/wrap (FP32), new cell key,
//                 rank within the cell.  Records of a block were sorted by
//                 their previous cell, so their new keys span a narrow range:
//                 ranks come from an LDS histogram and one global atomic per
//                 distinct key (global atomics per record as a fallback)
//   k_scan_*      exclusive prefix of the per-cell counts (and re-zero them)
//   k_scatter     record p -> its new cell-order position (ping-pong buffer),
//                 with its agent id and FP64 return; positions for the sweep
//   k_sweep       one lane per agent in the new cell order walks the cells of
//                 its (2r+1)^2 block (runs of consecutive cells, read from
//                 L2-resident sorted positions); per candidate: periodic
//                 image, d^2, radius tests, sector of the bearing, per-sector
//                 minimum in LDS; then view, reward and the FP64 return
//
// Envs of a batch live in one global cell space (env k's cells start at
// cell_base), so one counting sort serves every env and the cell-order range
// of env k equals its row range [agent_base, agent_base + n).
//
// Arithmetic contract (compiled with -ffp-contract=off):
//   * the move is IEEE FP32 operation by operation; cos/sin of the FP32
//     heading come from an FP32 evaluation within 1 ulp of the correctly
//     rounded values (heading_cs), so a new position is within one rounding
//     of the correctly rounded result of the stated operations;
//   * pair displacement: the periodic shift is applied to whichever operand
//     lies in the far half of the box, where the shift is exact, so dx and
//     dy carry a single rounding; d^2 = fma(dx, dx, dy*dy); the radius tests
//     are strict;
//   * the bearing comes from rotating (dx, dy) into the heading frame,
//     folding into the first octant and an odd polynomial for atan fitted
//     here (max error 3.4e-7 rad); with the FP32 roundings the sector
//     position is within about 1.5e-6 rad of the exact bearing;
//   * view: 1 - sqrt(d^2_min) * (1/R), within a few ulp of 1 - d_min/R.
#include <limits.h>

#include <algorithm>
#include <cmath>

#include <type_traits>

#include "flock_internal.h"

namespace flock {

namespace {

constexpr uint32_t kInfBits = 0x7f800000u;

// Positions lie in [0, L), so truncation is floor; the clamp keeps any
// out-of-range or NaN coordinate inside the grid (memory safety only).
__device__ __forceinline__ int cell_of(float v, float inv, int ncell) {
    int c = (int)(v * inv);
    c = c < ncell ? c : ncell - 1;
    return c > 0 ? c : 0;
}

// Last env e with base[e] <= row (skips empty envs, whose base equals the next).
__device__ __forceinline__ int env_search(const int32_t *base, int n_envs, int row) {
    int lo = 0, hi = n_envs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same search by the 64 lanes of one wave: each round splits [lo, hi)
// into 64 strides and keeps the last stride whose first base is <= row
// (base[lo] <= row holds throughout), so up to 64^k envs take k dependent
// loads instead of log2 of them.  Every lane of the wave must call it.
__device__ __forceinline__ int wave_env_search(const int32_t *base, int n_envs, int row) {
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n_envs;
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) >> 6;
        const int e = lo + lane * step;
        const bool ok = e < hi && base[e] <= row;
        const uint64_t m = __ballot(ok);  // lane 0 (e = lo) is always set
        lo += (63 - __builtin_clzll(m)) * step;
        hi = hi < lo + step ? hi : lo + step;
    }
    return lo;
}

constexpr bool kWaveSearch = true;

// Env of the block's first row into s_env (wave 0 searches).
__device__ __forceinline__ void block_env(int *s_env, const int32_t *base, int n_envs, int row) {
    if (kWaveSearch) {
        if (threadIdx.x < 64) {
            const int e = wave_env_search(base, n_envs, row);
            if (threadIdx.x == 0) *s_env = e;
        }
    } else if (threadIdx.x == 0) {
        *s_env = env_search(base, n_envs, row);
    }
}

__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d, 64));
    return x;
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x = max(x, __shfl_xor(x, d, 64));
    return x;
}

// Arrays reached through a DevEnv are device global memory, but a pointer
// read from memory is generic to the compiler, and it waits on generic
// accesses conservatively (they count as both vector-memory and LDS
// operations).  These access such arrays through the global address space.
// The sweep uses them where lane groups share an agent (its per-agent loads
// and stores then overlap better: 245 -> 230 us for 50k-agent blobs at four
// lanes); with one lane per agent the generic form measured faster.
#define FLOCK_GLOBAL __attribute__((address_space(1)))
typedef float gfloat4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ __forceinline__ T gload(const T *p, int64_t i) {
    return ((const FLOCK_GLOBAL T *)p)[i];
}

__device__ __forceinline__ float4 gload(const float4 *p, int64_t i) {
    const gfloat4 v = ((const FLOCK_GLOBAL gfloat4 *)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

template <class T>
__device__ __forceinline__ void gstore(T *p, int64_t i, T v) {
    ((FLOCK_GLOBAL T *)p)[i] = v;
}

// Either form, chosen at compile time.
template <bool kGlobal, class T>
__device__ __forceinline__ T load_as(const T *p, int64_t i) {
    if constexpr (kGlobal) return gload(p, i);
    else return p[i];
}

template <bool kGlobal, class T>
__device__ __forceinline__ void store_as(T *p, int64_t i, T v) {
    if constexpr (kGlobal) gstore(p, i, v);
    else p[i] = v;
}

// --------------------------------------------------------------------- move

constexpr int kHistBins = 2048;

// (cos h, sin h) of a heading in FP32 arithmetic.  Cody and Waite's
// additive range reduction (Software Manual for the Elementary Functions,
// 1980): k = nearest integer to h 2/pi, r = h - k pi/2 with pi/2 split into
// three FP32 parts and each product taken exactly inside an FMA, so r carries
// one rounding for |h| < 2^12; then odd / even polynomials in r^2 on
// [-pi/4, pi/4] (minimax fits made for this kernel: relative error 3.8e-9 for
// sin, absolute 9.6e-11 for cos) and the quadrant's swap and signs.  Checked
// on every FP32 heading in [0, 2pi_f]: within 1 ulp of the correctly rounded
// value, and correctly rounded for 99.4 % (cos) and 99.6 % (sin) of them
// (most FP32 values lie near 0); of headings drawn uniformly in value, 84 %
// and 94 %, the final rounding of r costing up to 0.35 ulp near pi/4.
__device__ __forceinline__ float2 heading_cs(float h) {
    const float k = __builtin_rintf(h * 0.636619772f);
    float r = __builtin_fmaf(-k, 1.57079637050628662109375f, h);
    r = __builtin_fmaf(-k, -4.37113882867379e-08f, r);
    r = __builtin_fmaf(-k, -1.7151245e-15f, r);
    const float z = r * r;
    float ps = __builtin_fmaf(z, -0.00019515264f, 0.008332161f);
    ps = __builtin_fmaf(z, ps, -0.16666655f);
    const float sn = __builtin_fmaf(r * z, ps, r);
    float pc = __builtin_fmaf(z, 2.4438208e-05f, -0.0013887365f);
    pc = __builtin_fmaf(z, pc, 0.041666646f);
    const float cs = __builtin_fmaf(z, __builtin_fmaf(z, pc, -0.5f), 1.0f);
    const int q = (int)k & 3;
    float c = (q & 1) ? sn : cs, s = (q & 1) ? cs : sn;
    c = (q == 1 || q == 2) ? -c : c;
    s = (q >= 2) ? -s : s;
    return make_float2(c, s);
}

// One agent's move (Sec. 4.1): turn, speed update (tag: the action is the
// speed), integrate with the new heading and speed, wrap into [0, L).
__device__ __forceinline__ float4 move_record(const DevEnv &E, float4 r, float2 av) {
    float x = r.x, y = r.y, h = r.z, sp = r.w;
    const float turn = fminf(fmaxf(av.x, -E.max_turn), E.max_turn);
    h = h + turn;
    if (h < 0.0f) h = h + kTwoPiF;
    if (h >= kTwoPiF) h = h - kTwoPiF;
    if (E.tag) {
        sp = fminf(fmaxf(av.y, 0.0f), E.s_max);
    } else {
        const float ds = fminf(fmaxf(av.y, -E.max_dspeed), E.max_dspeed);
        sp = fminf(fmaxf(sp + ds, E.s_min), E.s_max);
    }
    const float2 cs = heading_cs(h);
    const float c = cs.x, sn = cs.y;
    const float L = E.box;
    float nx = x + sp * c;
    if (nx < 0.0f) nx = nx + L;
    if (nx >= L) nx = nx - L;
    float ny = y + sp * sn;
    if (ny < 0.0f) ny = ny + L;
    if (ny >= L) ny = ny - L;
    return make_float4(nx, ny, h, sp);
}

// Cell of a position within its env's grid: column-major, rows within a column.
__device__ __forceinline__ int local_cell(const DevEnv &E, float x, float y) {
    return cell_of(x, E.inv_cx, E.ncx) * E.ncy + cell_of(y, E.inv_cy, E.ncy);
}

// Records per thread of the move kernel: a block covers kMoveRecs * kBlock
// consecutive records, all of whose loads are issued before any compute.
constexpr int kMoveRecs = 1;

__global__ __launch_bounds__(kBlock) void k_move_count(SortArrays a, const DevEnv *__restrict__ envs,
                                                       int n_envs, int G, int do_move,
                                                       const float2 *__restrict__ act,
                                                       float2 *__restrict__ act_copy) {
    constexpr int R = kMoveRecs;
    __shared__ int s_env;
    __shared__ int s_kmin[kBlock / 64], s_kmax[kBlock / 64];
    __shared__ int s_hist[kHistBins];
    const int p0 = blockIdx.x * (kBlock * R);
    block_env(&s_env, a.base, n_envs, p0);
    __syncthreads();
    // loads first: records, ids, then the actions they index
    int env[R], key[R];
    bool live[R];
    float4 rec[R];
    int id[R];
    float2 av[R];
    int e = s_env;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int p = p0 + r * kBlock + threadIdx.x;
        live[r] = p < G;
        key[r] = 0;
        env[r] = e;
        if (live[r]) {
            while (a.base[e + 1] <= p) ++e;
            env[r] = e;
            const DevEnv &E = envs[e];
            const int i = p - E.agent_base;
            rec[r] = E.rec_cur[i];
            id[r] = do_move ? E.id_cur[i] : 0;
        }
    }
    if (do_move) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!live[r]) continue;
            const DevEnv &E = envs[env[r]];
            if ((unsigned)id[r] >= (unsigned)E.n) continue;  // ids are agent indices (a guard)
            av[r] = act ? act[E.agent_base + id[r]] : reinterpret_cast<const float2 *>(E.act)[id[r]];
            if (act_copy) act_copy[E.agent_base + id[r]] = av[r];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!live[r]) continue;
        const int p = p0 + r * kBlock + threadIdx.x;
        const DevEnv &E = envs[env[r]];
        const float4 m = do_move ? move_record(E, rec[r], av[r]) : rec[r];
        a.tmp[p] = m;
        key[r] = E.cell_base + local_cell(E, m.x, m.y);
        a.key[p] = key[r];
    }
    // key range of the block
    int kmin = INT_MAX, kmax = INT_MIN;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        kmin = min(kmin, live[r] ? key[r] : INT_MAX);
        kmax = max(kmax, live[r] ? key[r] : INT_MIN);
    }
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_kmin[wid] = kmin;
        s_kmax[wid] = kmax;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        kmin = min(kmin, s_kmin[w]);
        kmax = max(kmax, s_kmax[w]);
    }
    const int range = kmax - kmin;  // >= 0: every block holds at least one record
    int slot[R];
    if (range < kHistBins) {
        for (int b = threadIdx.x; b <= range; b += kBlock) s_hist[b] = 0;
        __syncthreads();
        int lrank[R];
#pragma unroll
        for (int r = 0; r < R; ++r) lrank[r] = live[r] ? atomicAdd(&s_hist[key[r] - kmin], 1) : 0;
        __syncthreads();
        for (int b = threadIdx.x; b <= range; b += kBlock) {
            const int c = s_hist[b];
            if (c) s_hist[b] = atomicAdd(&a.count[kmin + b], c);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) slot[r] = live[r] ? s_hist[key[r] - kmin] + lrank[r] : 0;
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) slot[r] = live[r] ? atomicAdd(&a.count[key[r]], 1) : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (live[r]) a.slot[p0 + r * kBlock + threadIdx.x] = slot[r];
}

// --------------------------------------------------------------------- scan

// Exclusive block scan of one int per thread; also returns the block total.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int *s_wave, int *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    if (lane == 63) s_wave[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int w = lane < NT / 64 ? s_wave[lane] : 0;
        int wi = w;
#pragma unroll
        for (int d = 1; d < NT / 64; d <<= 1) {
            int t = __shfl_up(wi, d, 64);
            if (lane >= d) wi += t;
        }
        if (lane < NT / 64) s_wave[lane] = wi - w;
        if (lane == NT / 64 - 1) s_wave[NT / 64] = wi;
    }
    __syncthreads();
    const int r = s_wave[wid] + incl - v;
    *total = s_wave[NT / 64];
    return r;
}

constexpr int kScanNT = 1024;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanNT * kScanItems;  // cells of the single-block scan

// Every env has at most kScanTile cells: block e scans env e's cells on its
// own.  An env's agents occupy cell-order positions [agent_base, agent_base
// + n), so its cell starts are agent_base plus the prefix within the env;
// no block waits for another.  Re-zeroes the counts; the last env's block
// also writes start[C] (= the batch's agent total).
// NT threads of ITEMS cells each cover the largest env of the launch.
template <int NT, int ITEMS>
__global__ __launch_bounds__(NT) void k_scan_env(int32_t *__restrict__ count,
                                                 int32_t *__restrict__ start,
                                                 const DevEnv *__restrict__ envs, int n_envs, int C) {
    __shared__ int s_wave[NT / 64 + 1];
    __shared__ int s_tile[NT * ITEMS];
    const int t = threadIdx.x;
    const DevEnv &E = envs[blockIdx.x];
    const int cb = E.cell_base, Ce = E.ncx * E.ncy, base = E.agent_base;
    count += cb;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int idx = k * NT + t;  // coalesced: item-major
        s_tile[idx] = idx < Ce ? count[idx] : 0;
    }
    __syncthreads();
    int vals[ITEMS];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        vals[k] = s_tile[t * ITEMS + k];
        sum += vals[k];
    }
    int total;
    int run = block_exclusive_scan<NT>(sum, s_wave, &total) + base;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        s_tile[t * ITEMS + k] = run;
        run += vals[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int idx = k * NT + t;
        if (idx < Ce) {
            start[cb + idx] = s_tile[idx];
            count[idx] = 0;
        }
    }
    if (t == 0 && blockIdx.x == n_envs - 1) start[C] = base + total;
}

// Large C: tiles of kTile2 cells, one 256-thread block each.
constexpr int kScan2NT = 256;
constexpr int kScan2Items = 8;
constexpr int kTile2 = kScan2NT * kScan2Items;

// Phase 1: per-tile totals.  The phases are separate launches, whose
// boundaries order them; no block waits on another (a device-wide fence per
// block writes back an XCD's L2 and costs far more than a launch).
__global__ __launch_bounds__(kScan2NT) void k_tile_sums(const int32_t *__restrict__ count,
                                                        int32_t *__restrict__ part, int C) {
    __shared__ int s_wave[kScan2NT / 64 + 1];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile2;
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        const int64_t idx = base + k * kScan2NT + t;
        sum += idx < C ? count[idx] : 0;
    }
    int total;
    (void)block_exclusive_scan<kScan2NT>(sum, s_wave, &total);
    if (t == 0) part[blockIdx.x] = total;
}

// Up to this many tiles, each tile of phase 2 sums the totals before it
// itself; beyond, one block first turns them into exclusive offsets.
constexpr int kDirectTiles = 4096;

// Phase 1b (more than kDirectTiles tiles): one block, exclusive offsets of
// the nb tile totals in place, in chunks of kTile2 with a running carry.
__global__ __launch_bounds__(kScan2NT) void k_scan_parts(int32_t *__restrict__ part, int nb) {
    __shared__ int s_wave[kScan2NT / 64 + 1];
    const int t = threadIdx.x;
    int carry = 0;
    for (int c0 = 0; c0 < nb; c0 += kTile2) {
        int vals[kScan2Items];
        int psum = 0;
#pragma unroll
        for (int k = 0; k < kScan2Items; ++k) {
            const int idx = c0 + t * kScan2Items + k;
            vals[k] = idx < nb ? part[idx] : 0;
            psum += vals[k];
        }
        int chunk;
        int run = block_exclusive_scan<kScan2NT>(psum, s_wave, &chunk) + carry;
#pragma unroll
        for (int k = 0; k < kScan2Items; ++k) {
            const int idx = c0 + t * kScan2Items + k;
            if (idx < nb) part[idx] = run;
            run += vals[k];
        }
        carry += chunk;
        __syncthreads();  // s_wave is reused by the next chunk
    }
}

// Phase 2: scan each tile from its offset; re-zero the counts.  kSum: the
// offset is the sum of the totals of the tiles before (at most kDirectTiles
// of them), else part holds the offsets.  The last tile writes start[C].
template <bool kSum>
__global__ __launch_bounds__(kScan2NT) void k_scan_down(int32_t *__restrict__ count,
                                                        const int32_t *__restrict__ part,
                                                        int32_t *__restrict__ start, int C) {
    __shared__ int s_wave[kScan2NT / 64 + 1];
    __shared__ int s_tile[kTile2];
    __shared__ int s_off;
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile2;
    if constexpr (kSum) {
        int before = 0;
        for (int b = t; b < (int)blockIdx.x; b += kScan2NT) before += part[b];
        int sum_before;
        (void)block_exclusive_scan<kScan2NT>(before, s_wave, &sum_before);
        if (t == 0) s_off = sum_before;
    } else {
        if (t == 0) s_off = part[blockIdx.x];
    }
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        const int64_t idx = base + k * kScan2NT + t;
        s_tile[k * kScan2NT + t] = idx < C ? count[idx] : 0;
    }
    __syncthreads();
    int vals[kScan2Items];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        vals[k] = s_tile[t * kScan2Items + k];
        sum += vals[k];
    }
    int total;
    const int off = s_off;  // published before the scan's barriers
    int run = block_exclusive_scan<kScan2NT>(sum, s_wave, &total) + off;
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        s_tile[t * kScan2Items + k] = run;
        run += vals[k];
    }
    if (t == 0 && blockIdx.x == gridDim.x - 1) start[C] = off + total;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScan2Items; ++k) {
        const int64_t idx = base + k * kScan2NT + t;
        if (idx < C) {
            start[idx] = s_tile[k * kScan2NT + t];
            count[idx] = 0;
        }
    }
}

// --------------------------------------------------- per-env fused sort

// Batches of many envs that each fit one block: block e moves env e's
// agents, counts them per cell in LDS, scans its own cells and scatters the
// records into the new cell order -- the move, count, scan and scatter of
// the separate kernels in one launch, with no global atomics.  Ranks within
// a cell come from LDS atomics, so the order inside a cell varies from run
// to run; every output is independent of that order.  Up to R records per
// thread; the env's cell counts, then starts, live in dynamic LDS.  Up to
// kEnvRegR records per thread the moved records and ids wait in registers
// for the scatter; above that they are staged in `tmp`.
constexpr int kEnvNT = 1024;
constexpr int kEnvRegR = 8;

template <int R>
__global__ __launch_bounds__(kEnvNT) void k_env_sort(SortArrays a, const DevEnv *__restrict__ envs,
                                                     int n_envs, int C, int do_move,
                                                     const float2 *__restrict__ act, int tag,
                                                     float2 *__restrict__ act_copy) {
    extern __shared__ int s_cells[];  // [Ce] counts, then starts within the env
    __shared__ int s_wave[kEnvNT / 64 + 1];
    const int tid = threadIdx.x;
    const DevEnv &E = envs[blockIdx.x];
    const int n = E.n, base = E.agent_base, cb = E.cell_base, Ce = E.ncx * E.ncy;
    for (int c = tid; c < Ce; c += kEnvNT) s_cells[c] = 0;
    __syncthreads();
    constexpr bool kRegs = R <= kEnvRegR;
    constexpr int RR = kRegs ? R : 1;
    int key[R], rank[R];
    float4 mr[RR];
    int idr[RR];
    double retr[RR];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kEnvNT + tid;
        key[r] = 0;
        rank[r] = 0;
        if (i < n) {
            float4 m = E.rec_cur[i];
            const int id = E.id_cur[i];
            if (do_move) {
                float2 av = make_float2(0.0f, 0.0f);
                if ((unsigned)id < (unsigned)n) {  // ids are agent indices (a guard)
                    av = act ? act[base + id] : reinterpret_cast<const float2 *>(E.act)[id];
                    if (act_copy) act_copy[base + id] = av;
                }
                m = move_record(E, m, av);
            }
            if constexpr (kRegs) {
                mr[r] = m;
                idr[r] = id;
                retr[r] = E.ret_cur[i];  // loaded now, stored after the scan
            } else {
                a.tmp[base + i] = m;
            }
            key[r] = local_cell(E, m.x, m.y);
            rank[r] = atomicAdd(&s_cells[key[r]], 1);
        }
    }
    __syncthreads();
    // exclusive scan of the counts: thread t owns cells [t k, t k + k)
    const int per = (Ce + kEnvNT - 1) / kEnvNT;
    const int c0 = tid * per;
    int sum = 0;
    for (int c = c0; c < c0 + per && c < Ce; ++c) sum += s_cells[c];
    int total;
    int run = block_exclusive_scan<kEnvNT>(sum, s_wave, &total);
    for (int c = c0; c < c0 + per && c < Ce; ++c) {
        const int cnt = s_cells[c];
        s_cells[c] = run;
        run += cnt;
    }
    if (tid == 0 && blockIdx.x == n_envs - 1) a.start[C] = base + n;
    __syncthreads();
    for (int c = tid; c < Ce; c += kEnvNT) a.start[cb + c] = base + s_cells[c];  // coalesced
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * kEnvNT + tid;
        if (i < n) {
            const int j = s_cells[key[r]] + rank[r];
            float4 m;
            int id;
            double ret;
            if constexpr (kRegs) {
                m = mr[r];
                id = idr[r];
                ret = retr[r];
            } else {
                m = a.tmp[base + i];
                id = E.id_cur[i];
                ret = E.ret_cur[i];
            }
            E.rec_nxt[j] = m;
            E.id_nxt[j] = id;
            E.ret_nxt[j] = ret;
            a.sxy[base + j] = make_float2(m.x, m.y);
            if (tag) a.stype[base + j] = id < E.n_chasers ? 1 : 0;
        }
    }
}

// ------------------------------------------------------------- strip sort

// One block per strip of columns of one env (see carve_sort and the plan's
// strips in flock_internal.h).  The records are in cell order (column
// major), so the records of a range of columns are one range of records,
// found by a search; an agent moves at most one column per step, so the
// agents now in the strip were, before the move, in its columns or in the one
// on either side.  The block moves those (twice: once to count, once to
// place, reading the records again from cache instead of keeping a variable
// number of them), ranks its agents by cell in LDS, takes its first output
// row from the strips of the env before it by decoupled look-back, and
// writes its agents in cell order and its cells' starts.
constexpr int kStripNT = 512;
constexpr int kXcds = 8;     // MI355X: accelerator dies (XCDs), each with its own L2
constexpr int kStripR = 4;   // old records per thread and round (placing by a second pass)
constexpr int kStripR1 = 4;  // old records per thread and round of the counting pass (8: no faster, 89 VGPRs)
constexpr uint32_t kStripAgg = 1u << 30;   // look-back word: the strip's own count is set
constexpr uint32_t kStripIncl = 1u << 31;  // the count of the env's strips up to this one is set
constexpr uint32_t kStripVal = kStripAgg - 1;
// Look-back waits are bounded (the plan's strip_wait polling rounds).  With
// tickets a strip waits only for strips already running.  Without them (the
// block index picks the strip) every block is meant to be resident at once,
// which the runtime's occupancy figure suggests but nothing guarantees: a
// strip whose wait runs out counts the agents before it itself
// (strip_base_by_count), so the sort stays exact and the wait bounded.

// The env's agents that the step moves into columns below c0: every old
// record of env E moved as in the strip sort (one wave, all of its lanes
// calling).  The look-back's fallback, O(n) per call.
__device__ int strip_base_by_count(const DevEnv &E, int c0, int do_move,
                                   const float2 *__restrict__ act) {
    const int lane = threadIdx.x & 63;
    int cnt = 0;
    for (int i = lane; i < E.n; i += 64) {
        float4 m = E.rec_cur[i];
        if (do_move) {
            const int id = E.id_cur[i];
            float2 av = make_float2(0.0f, 0.0f);
            if ((unsigned)id < (unsigned)E.n)
                av = act ? act[E.agent_base + id] : reinterpret_cast<const float2 *>(E.act)[id];
            m = move_record(E, m, av);
        }
        cnt += cell_of(m.x, E.inv_cx, E.ncx) < c0 ? 1 : 0;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    return cnt;
}

// First record of env E (cell order) whose column is >= col; n when col >=
// ncx.  Every lane of the calling wave takes part: each round probes 64
// evenly spaced records of the remaining range (columns are nondecreasing, so
// the probes below col form a prefix of the lanes).
__device__ int wave_first_col(const DevEnv &E, int col) {
    if (col <= 0) return 0;
    if (col >= E.ncx) return E.n;
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = E.n;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int step = (hi - lo + 63) >> 6;
        const int q = lo + lane * step;
        const bool below = q < hi && cell_of(E.rec_cur[q].x, E.inv_cx, E.ncx) < col;
        const uint64_t m = __ballot(below);
        const int k = m ? 64 - __builtin_clzll(m) : 0;  // probes below col
        if (k == 0) break;                              // record lo is at or past col
        const int next = lo + k * step;                 // first probe not below (or past hi)
        lo = lo + (k - 1) * step + 1;
        hi = next < hi ? next : hi;
    }
    return lo;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_strip_sort(SortArrays a, const DevEnv *__restrict__ envs,
                                                   int n_envs, int C, int G, int S, int do_move,
                                                   const float2 *__restrict__ act, int tag,
                                                   float2 *__restrict__ act_copy, int cap,
                                                   int direct, int wait) {
    // dynamic LDS: the strip's cells (counts, then each cell's next free row),
    // then up to `cap` of its agents: old record, cell, action
    extern __shared__ int s_dyn[];
    __shared__ int s_wave[NT / 64 + 1];
    __shared__ int s_tk, s_base, s_own;
    __shared__ int s_rng[4];
    const int tid = threadIdx.x;
    if (tid == 0) {
        // With few strips every block is resident at once and the block index
        // picks the strip: blocks go to the XCDs round robin, and XCD x takes
        // the x-th run of `direct` consecutive strips, so an env's strips share
        // one or two XCDs' L2 for their action gathers.  Otherwise a ticket
        // makes strips start in order.
        if (direct) {
            const int x = (int)blockIdx.x % kXcds, k = (int)blockIdx.x / kXcds;
            s_tk = k < direct ? x * direct + k : S;
        } else {
            s_tk = (int)atomicAdd(&a.status[S], 1u);
        }
        s_own = 0;
    }
    __syncthreads();
    const int t = s_tk;
    if (t >= S) return;  // a block past the last strip (direct mode padding)
    const DevEnv &E = envs[n_envs == 1 ? 0 : a.strip_env[t]];
    const int ls = t - E.strip_base, nst = E.n_strips, ncx = E.ncx, ncy = E.ncy, n = E.n;
    const int c0 = ls * E.strip_cols, c1 = ls == nst - 1 ? ncx : c0 + E.strip_cols;
    const int cbase = c0 * ncy, ncell = (c1 - c0) * ncy;
    int *s_cells = s_dyn;
    int *s_oi = s_dyn + ((ncell + 3) & ~3);
    int *s_oc = s_oi + cap;
    float2 *s_oa = reinterpret_cast<float2 *>(s_oc + cap);
    for (int c = tid; c < ncell; c += NT) s_cells[c] = 0;
    // old records of columns c0 - 1 .. c1 (periodic): all of them when those
    // columns cover the box, else one range or two (wrapping); waves 0 and 1
    // search one boundary each
    if (tid == 0) {
        s_rng[0] = 0;
        s_rng[1] = n;
        s_rng[2] = 0;
        s_rng[3] = 0;
    }
    __syncthreads();
    if (nst > 1 && c1 - c0 + 2 < ncx && tid < 128) {
        const int w = tid >> 6;
        int col, slot;
        if (c0 == 0) {
            col = w == 0 ? ncx - 1 : c1 + 1;
            slot = w == 0 ? 0 : 3;
        } else if (c1 == ncx) {
            col = w == 0 ? c0 - 1 : 1;
            slot = w == 0 ? 0 : 3;
        } else {
            col = w == 0 ? c0 - 1 : c1 + 1;
            slot = w == 0 ? 0 : 1;
        }
        const int r = wave_first_col(E, col);
        if ((tid & 63) == 0) s_rng[slot] = r;
    }
    __syncthreads();
    // kStripR old records per thread and round, all loads issued before any
    // is used (each record's action is a gather by its id); each record is
    // moved as in k_env_sort
    constexpr int R = kStripR;
    auto round = [&](int i0, int i1, auto use) {
        int id[R];
        float4 m[R];
        float2 av[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = i0 + u * NT;
            id[u] = i < i1 ? E.id_cur[i] : 0;
            m[u] = i < i1 ? E.rec_cur[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = i0 + u * NT;
            av[u] = make_float2(0.0f, 0.0f);
            if (do_move && i < i1 && (unsigned)id[u] < (unsigned)E.n)
                av[u] = act ? act[E.agent_base + id[u]]
                            : reinterpret_cast<const float2 *>(E.act)[id[u]];
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int i = i0 + u * NT;
            if (i >= i1) continue;
            const float4 mm = do_move ? move_record(E, m[u], av[u]) : m[u];
            const int cx = cell_of(mm.x, E.inv_cx, ncx);
            if (cx >= c0 && cx < c1)
                use(i, mm, id[u], av[u], cx * ncy + cell_of(mm.y, E.inv_cy, ncy) - cbase);
        }
    };
    auto each_old = [&](auto use) {
        for (int r = 0; r < 4; r += 2)
            for (int i0 = s_rng[r] + tid; i0 < s_rng[r + 1]; i0 += R * NT)
                round(i0, s_rng[r + 1], use);
    };
    // pass 1: count the strip's agents per cell, listing the first `cap` of
    // them (one LDS atomic per wave and record slot for the list position);
    // kStripR1 records per thread and round
    const int lane = tid & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    constexpr int R1 = kStripR1;
    for (int r = 0; r < 4; r += 2)
        for (int i0 = s_rng[r] + tid; i0 < s_rng[r + 1]; i0 += R1 * NT) {
            const int i1 = s_rng[r + 1];
            int id[R1];
            float4 m[R1];
            float2 av[R1];
#pragma unroll
            for (int u = 0; u < R1; ++u) {
                const int i = i0 + u * NT;
                id[u] = i < i1 ? E.id_cur[i] : 0;
                m[u] = i < i1 ? E.rec_cur[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < R1; ++u) {
                const int i = i0 + u * NT;
                av[u] = make_float2(0.0f, 0.0f);
                if (do_move && i < i1 && (unsigned)id[u] < (unsigned)E.n)
                    av[u] = act ? act[E.agent_base + id[u]]
                                : reinterpret_cast<const float2 *>(E.act)[id[u]];
            }
#pragma unroll
            for (int u = 0; u < R1; ++u) {
                const int i = i0 + u * NT;
                int cell = -1;
                if (i < i1) {
                    const float4 mm = do_move ? move_record(E, m[u], av[u]) : m[u];
                    const int cx = cell_of(mm.x, E.inv_cx, ncx);
                    if (cx >= c0 && cx < c1) cell = cx * ncy + cell_of(mm.y, E.inv_cy, ncy) - cbase;
                }
                const uint64_t mask = __ballot(cell >= 0);
                if (mask == 0) continue;
                const int leader = __builtin_ctzll(mask);
                int wbase = 0;
                if (lane == leader) wbase = atomicAdd(&s_own, __popcll(mask));
                wbase = __shfl(wbase, leader, 64);
                if (cell >= 0) {
                    atomicAdd(&s_cells[cell], 1);
                    const int k = wbase + __popcll(mask & below);
                    if (k < cap) {
                        s_oi[k] = i;
                        s_oc[k] = cell;
                        s_oa[k] = av[u];
                    }
                }
            }
        }
    __syncthreads();
    // exclusive scan of the counts: thread t owns cells [t k, t k + k)
    const int per = (ncell + NT - 1) / NT;
    const int q0 = tid * per;
    int sum = 0;
    for (int c = q0; c < q0 + per && c < ncell; ++c) sum += s_cells[c];
    int total;
    int run = block_exclusive_scan<NT>(sum, s_wave, &total);
    for (int c = q0; c < q0 + per && c < ncell; ++c) {
        const int cnt = s_cells[c];
        s_cells[c] = run;
        run += cnt;
    }
    if (tid < 64) {
        // the env's agents before this strip: decoupled look-back over the
        // env's earlier strips, 64 of them per round (lane k reads strip
        // t - 1 - k): the counts down to the nearest strip whose running total
        // is set, once every one of them has published
        uint32_t *st = a.status;
        const int lane = tid;
        int base = 0;
        if (ls == 0) {
            if (lane == 0)
                __hip_atomic_store(&st[t], kStripIncl | (uint32_t)total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&st[t], kStripAgg | (uint32_t)total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            int top = t - 1, spins = 0;
            while (spins < wait) {
                const int j = top - lane;
                const bool valid = j >= E.strip_base;
                const uint32_t w = valid ? __hip_atomic_load(&st[j], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)
                                         : 0u;
                const uint64_t incl = __ballot(valid && (w & kStripIncl));
                const uint64_t ready = __ballot(valid && (w & (kStripIncl | kStripAgg)));
                const uint64_t need = incl ? (incl & (~incl + 1)) * 2 - 1  // lanes up to the nearest total
                                           : __ballot(valid);
                if ((ready & need) != need) {
                    ++spins;
                    continue;
                }
                int v = ((need >> lane) & 1) ? (int)(w & kStripVal) : 0;
#pragma unroll
                for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
                base += v;
                if (incl) break;
                top -= 64;
            }
            if (spins >= wait) base = strip_base_by_count(E, c0, do_move, act);
            if (lane == 0)
                __hip_atomic_store(&st[t], kStripIncl | (uint32_t)(base + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_base = base;
            if (t == S - 1) a.start[C] = G;
        }
    }
    __syncthreads();
    const int base = s_base;
    for (int c = tid; c < ncell; c += NT) a.start[E.cell_base + cbase + c] = E.agent_base + base + s_cells[c];
    __syncthreads();  // the starts are read before the counts become row cursors
    // place the strip's agents: from the list (one load round: record, id,
    // return), or, when the strip holds more than `cap`, by a second pass
    auto place = [&](int i, const float4 &m, int id, float2 av, int cell) {
        const int j = base + atomicAdd(&s_cells[cell], 1);
        E.rec_nxt[j] = m;
        E.id_nxt[j] = id;
        E.ret_nxt[j] = E.ret_cur[i];
        a.sxy[E.agent_base + j] = make_float2(m.x, m.y);
        if (tag) a.stype[E.agent_base + j] = id < E.n_chasers ? 1 : 0;
        if (do_move && act_copy && (unsigned)id < (unsigned)E.n) act_copy[E.agent_base + id] = av;
    };
    const int own = s_own;
    if (own <= cap) {
        for (int k0 = tid; k0 < own; k0 += R * NT) {
            int oi[R], id[R];
            float4 m[R];
            double ret[R];
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int k = k0 + u * NT;
                oi[u] = k < own ? s_oi[k] : 0;
                id[u] = k < own ? E.id_cur[oi[u]] : 0;
                m[u] = k < own ? E.rec_cur[oi[u]] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                ret[u] = k < own ? E.ret_cur[oi[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int k = k0 + u * NT;
                if (k >= own) continue;
                const float2 av = s_oa[k];
                const float4 mm = do_move ? move_record(E, m[u], av) : m[u];
                const int j = base + atomicAdd(&s_cells[s_oc[k]], 1);
                E.rec_nxt[j] = mm;
                E.id_nxt[j] = id[u];
                E.ret_nxt[j] = ret[u];
                a.sxy[E.agent_base + j] = make_float2(mm.x, mm.y);
                if (tag) a.stype[E.agent_base + j] = id[u] < E.n_chasers ? 1 : 0;
                if (do_move && act_copy && (unsigned)id[u] < (unsigned)E.n)
                    act_copy[E.agent_base + id[u]] = av;
            }
        }
    } else {
        each_old(place);
    }
}

// ------------------------------------------------------------------ scatter

__global__ __launch_bounds__(kBlock) void k_scatter(SortArrays a, const DevEnv *__restrict__ envs,
                                                    int n_envs, int G, int tag) {
    __shared__ int s_env;
    const int p0 = blockIdx.x * kBlock;
    block_env(&s_env, a.base, n_envs, p0);
    __syncthreads();
    const int p = p0 + threadIdx.x;
    if (p >= G) return;
    int e = s_env;
    while (a.base[e + 1] <= p) ++e;
    const DevEnv &E = envs[e];
    const int i = p - E.agent_base;
    const int pos = a.start[a.key[p]] + a.slot[p];
    const int j = pos - E.agent_base;
    const float4 r = a.tmp[p];
    const int id = E.id_cur[i];
    E.rec_nxt[j] = r;
    E.id_nxt[j] = id;
    E.ret_nxt[j] = E.ret_cur[i];
    a.sxy[pos] = make_float2(r.x, r.y);
    if (tag) a.stype[pos] = id < E.n_chasers ? 1 : 0;
}

// -------------------------------------------------------------------- sweep

// atan(t) / (2 pi) for t in [0, 1] as t * P(t^2); least-squares fit with
// minimax reweighting on Chebyshev nodes, max error 5.4e-8 turns.
__device__ __forceinline__ float atan_turns01(float t) {
    const float t2 = t * t;
    float p = 0.0010841276962310076f;
    p = __builtin_fmaf(t2, p, -0.005348269362002611f);
    p = __builtin_fmaf(t2, p, 0.012672491371631622f);
    p = __builtin_fmaf(t2, p, -0.02106151357293129f);
    p = __builtin_fmaf(t2, p, 0.03152511641383171f);
    p = __builtin_fmaf(t2, p, -0.0530262365937233f);
    p = __builtin_fmaf(t2, p, 0.15915432572364807f);
    return p * t;
}

// Sector of the bearing of (dx, dy) relative to the heading (c, s): sector 0
// starts at the heading, sectors run counter-clockwise; (0, 0) -> sector 0.
__device__ __forceinline__ int sector_of(float dx, float dy, float c, float s, float vf, int v) {
    const float u = __builtin_fmaf(dx, c, dy * s);      // along the heading
    const float w = __builtin_fmaf(dy, c, -(dx * s));   // to its left
    const float au = fabsf(u), aw = fabsf(w);
    const float mx = fmaxf(au, aw), mn = fminf(au, aw);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    float a = atan_turns01(t);
    a = aw > au ? 0.25f - a : a;
    a = u < 0.0f ? 0.5f - a : a;
    a = w < 0.0f ? 1.0f - a : a;
    const int k = (int)(a * vf);
    return k < v - 1 ? k : v - 1;
}

// As sector_of for a full view with v = 8 M sectors (M sectors per octant),
// without the arctangent: the octant comes from the signs and the larger of
// |u| and |w|, the sector within it from comparing min/max with the
// tangents of the octant's interior sector edges, and mirrored octants
// count their sectors backwards.  A bearing exactly on an octant edge may
// land in either neighbouring sector (both are within the ambiguity band).
template <int M>
__device__ __forceinline__ int sector_oct(float dx, float dy, float c, float s) {
    const float u = __builtin_fmaf(dx, c, dy * s);
    const float w = __builtin_fmaf(dy, c, -(dx * s));
    const float au = fabsf(u), aw = fabsf(w);
    // min/max > tan(edge), tested as min > tan(edge) * max (no division; a
    // coincident pair, max = 0, stays in sector 0)
    int j = 0;
    if constexpr (M > 1) {
        const float mx = fmaxf(au, aw), mn = fminf(au, aw);
        if constexpr (M == 2) {
            j = mn > 0.41421356237309503f * mx ? 1 : 0;  // tan(pi/8)
        } else {
            static_assert(M == 4, "sector_oct takes M = 1, 2 or 4");
            j = (mn > 0.19891236737965800f * mx ? 1 : 0) + (mn > 0.41421356237309503f * mx ? 1 : 0) +
                (mn > 0.66817863791929891f * mx ? 1 : 0);  // tan(pi/16), tan(pi/8), tan(3 pi/16)
        }
    }
    // mirroring within [0, 2^b) is an XOR with 2^b - 1, so the three mirrors
    // (past 45 degrees, past 90, past 180) flip whole bit groups: the top bit
    // is w < 0, the next (u < 0) ^ (w < 0), the lower ones that ^ (|w| > |u|),
    // and j's bits flip with those (kept as lane masks, combined once)
    const bool b3 = w < 0.0f;
    const bool b2 = b3 ^ (u < 0.0f);
    const bool b1 = b2 ^ (aw > au);
    if constexpr (M == 1) {
        return (b3 ? 4 : 0) | (b2 ? 2 : 0) | (b1 ? 1 : 0);
    } else if constexpr (M == 2) {
        return (b3 ? 8 : 0) | (b2 ? 4 : 0) | (b1 ? 2 : 0) | ((b1 ^ (j != 0)) ? 1 : 0);
    } else {
        return (b3 ? 16 : 0) | (b2 ? 8 : 0) | (b1 ? 4 : 0) | (j ^ (b1 ? 3 : 0));
    }
}

// View sector of the bearing of (dx, dy) for a limited field of view: the
// bearing in turns from the heading (as in sector_of), shifted by half the
// arc and wrapped, is seen iff it lies in the arc; -1 when not seen.  A
// coincident agent counts as straight ahead: the middle sector v/2.
__device__ __forceinline__ int view_sector(float dx, float dy, float c, float s, float fov_half,
                                           float fov_t, float sec_scale, int v) {
    const float u = __builtin_fmaf(dx, c, dy * s);
    const float w = __builtin_fmaf(dy, c, -(dx * s));
    const float au = fabsf(u), aw = fabsf(w);
    const float mx = fmaxf(au, aw), mn = fminf(au, aw);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    float a = atan_turns01(t);
    a = aw > au ? 0.25f - a : a;
    a = u < 0.0f ? 0.5f - a : a;
    a = w < 0.0f ? 1.0f - a : a;
    float p = a + fov_half;
    p = p >= 1.0f ? p - 1.0f : p;
    int k = (int)(p * sec_scale);
    k = p < fov_t ? (k < v - 1 ? k : v - 1) : -1;
    return mx > 0.0f ? k : (v >> 1);
}

// Periodic displacement for single-cell (all-pairs) envs: the shift by L is
// applied to whichever operand lies in the far half, where it is exact.
__device__ __forceinline__ float min_image_delta(float xj, float xi, float L) {
    const float d = xj - xi;
    if (d > 0.5f * L) return (xj - L) - xi;
    if (d < -0.5f * L) return xj - (xi - L);
    return d;
}

// View constants of the lane's agent (see DevEnv).
struct ViewK {
    float c, s;                       // cos / sin of the heading
    float fov_half, fov_t, sec_scale;
    float vf;
    int v;
};

// Test candidate qq against the lane's agent (ok: the slot holds a candidate
// other than the agent itself): distance test, and for a
// neighbour the count, the collision count and the per-sector minimum (an
// LDS atomic min on the agent's own minima, S words apart).  The sector is
// computed for every candidate (branch-free); only the LDS update is
// predicated.  With G lanes per agent, lane li takes candidates q + li,
// q + li + G, ...  (offx, xi), (offy, yi): candidate shift (0 or -L) and
// centre (x or x - L) per axis; minimg selects the per-candidate minimum
// image (single-cell envs).  kFov selects the limited-view sector
// (candidates outside the arc are counted but update no sector).
//
// kTag (tag environment): candidate q's type stype[q] picks the view channel
// (minima at smin_own[(tj v + k) S]); nb counts runners in range and col
// touches with the other type (the lane's own type is ti).
// kShiftX / kShiftY: the candidate-side shift offx / offy may be nonzero (a
// zero shift is left out: x + 0 = x for the nonnegative coordinates here).
template <int S, bool kFov, bool kTag, int kM, bool kShiftX, bool kShiftY>
__device__ __forceinline__ void test_pair(uint32_t *smin_own, const uint8_t *__restrict__ stype,
                                          int ti, const float2 pj, int qq, bool ok, float offx,
                                          float xi, float offy, float yi, bool minimg, float L,
                                          float r2, float c2, const ViewK &K, int &nb, int &col) {
    float dx, dy;
    if (minimg) {
        dx = min_image_delta(pj.x, xi, L);
        dy = min_image_delta(pj.y, yi, L);
    } else {
        dx = (kShiftX ? pj.x + offx : pj.x) - xi;
        dy = (kShiftY ? pj.y + offy : pj.y) - yi;
    }
    const float d2 = __builtin_fmaf(dx, dx, dy * dy);
    const bool nbr = ok && d2 < r2;
    int ch = 0;  // view channel offset (sectors)
    if constexpr (kTag) {
        const int tj = stype[qq];
        nb += (nbr && tj == 0) ? 1 : 0;
        col += (nbr && tj != ti && d2 < c2) ? 1 : 0;
        ch = tj * K.v;
    } else if constexpr (kFov) {
        nb += nbr ? 1 : 0;
        col += (nbr && d2 < c2) ? 1 : 0;
    }
    if (kFov) {
        const int k = view_sector(dx, dy, K.c, K.s, K.fov_half, K.fov_t, K.sec_scale, K.v);
        if (nbr && k >= 0) atomicMin(&smin_own[(ch + k) * S], __float_as_uint(d2));
    } else {
        int k;
        if constexpr (kM > 0) k = sector_oct<kM>(dx, dy, K.c, K.s);
        else k = sector_of(dx, dy, K.c, K.s, K.vf, K.v);
        if (nbr) {
            // full view: the counts go with the neighbour's branch, which some
            // lane of the wave takes on nearly every slot anyway
            if constexpr (!kTag) {
                ++nb;
                if (d2 < c2) ++col;
            }
            atomicMin(&smin_own[(ch + k) * S], __float_as_uint(d2));
        }
    }
}

template <int S, int G, int UNROLL, bool kFov, bool kTag, int kM, bool kShiftX, bool kShiftY>
__device__ __forceinline__ void sweep_run(uint32_t *smin_own, const float2 *__restrict__ sxy,
                                          const uint8_t *__restrict__ stype, int ti,
                                          int q, int q1, int li, int self, float offx, float xi,
                                          float offy, float yi, bool minimg, float L, float r2,
                                          float c2, const ViewK &K, int &nb, int &col) {
    auto test = [&](const float2 pj, int qq, bool valid) {
        test_pair<S, kFov, kTag, kM, kShiftX, kShiftY>(smin_own, stype, ti, pj, qq,
                                                       valid && qq != self, offx, xi, offy, yi,
                                                       minimg, L, r2, c2, K, nb, col);
    };
    // UNROLL candidates per lane and step, those past the run's end masked
    // (the position arrays are padded for the reads)
    for (q += li; q < q1; q += UNROLL * G) {
        float2 pj[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) pj[u] = sxy[q + u * G];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) test(pj[u], q + u * G, q + u * G < q1);
    }
}

// Rows [lo, hi] of the column ox columns from the agent's own that can hold
// a point within the vision radius: the column's nearest x lies dmin from
// the agent, so only |dy| < sqrt(R^2 - dmin^2) matters.  fx is the agent's
// offset within its own column.  Both bounds widen by E.marg, which covers
// the FP32 rounding of the row assignment, of these bounds and of the pair
// test.  hi - lo < ncy; lo < 0 or hi >= ncy wrap through the column's ends.
// False when no point of the column is within the radius.
struct RowGeom {
    float cw, marg, r2, inv_cy;
    int ncy;
};

__device__ __forceinline__ bool column_rows(const RowGeom &E, float fx, int ox, float y, int &lo,
                                            int &hi) {
    float dmin = 0.0f;
    if (ox < 0) dmin = fx + (float)(-ox - 1) * E.cw;
    else if (ox > 0) dmin = (E.cw - fx) + (float)(ox - 1) * E.cw;
    dmin = fmaxf(dmin - E.marg, 0.0f);
    const float e2 = E.r2 - dmin * dmin;
    if (!(e2 > 0.0f)) return false;
    const float ext = __builtin_amdgcn_sqrtf(e2) + E.marg;  // within 1 ulp
    const int n = E.ncy;
    int l = (int)floorf((y - ext) * E.inv_cy);
    int h = (int)floorf((y + ext) * E.inv_cy);
    // in range for finite positions in [0, L); the clamps keep any other
    // input inside the column (memory safety only)
    l = max(min(l, n - 1), -n);
    h = max(min(h, l + n - 1), l);
    lo = l;
    hi = h;
    return true;
}

// Candidates per lane and loop step of a lane group's run (independent loads
// in flight): groups of 16 or 64 lanes split a run into short pieces, where
// masked slots past its end cost more than fewer loads in flight (MI355X,
// 128-sector flock at 16 lanes: 209 us at 4, 193 at 2; 4 lanes: 242 at 4,
// 248 at 2).
template <int G>
constexpr int unroll_for() { return G >= 16 ? 2 : 4; }
constexpr int kUnrollMax = 4;
// One lane per agent, stencil half-width 1: walk the agent's runs as one
// sequence (a lane moves to its next run as soon as its current one ends)
// instead of run by run, so a wave waits for its longest total rather than
// for the longest lane of every run.  The runs are found once per agent and
// queued in registers: lanes switch runs at different steps, so whatever a
// switch costs is paid by the whole wave on nearly every step.
constexpr bool kFlatRuns = true;
// Candidates per step of the flat walk; step of 200 x 5,000 agents, 16 sectors:
// 4 -> 70.1 us, 5 -> 71.0, 6 -> 70.6, 8 -> 73.2.
constexpr int kFlatUnroll = 4;
// Entries past the end of the cell-order position and type arrays, so that a
// step's reads past the last run stay inside the allocation: a lane reads at
// most (unroll - 1) * G + G - 1 < kUnrollMax * 64 (lane groups of G <= 64)
// or kFlatUnroll - 1 entries past its run's end.
constexpr int kSortPad = 256;
static_assert(unroll_for<4>() <= kUnrollMax && unroll_for<64>() <= kUnrollMax, "unroll bound");
static_assert(kFlatUnroll <= kSortPad + 1 && kUnrollMax * 64 <= kSortPad + 1,
              "pad the cell-order arrays for the unrolled reads");

// The runs of one agent's flat walk (one lane per agent, one column either
// side), for an agent at (fx into its column cx, y): slot c (c < 3) holds
// column cx + c - 1's first segment, slot 3 + c its second (empty unless the
// rows wrap), each as [rq, rq1) in cell order, with 4 bits of shift flags per
// slot in fl (1 candidate x - L, 2 centre x - L, 4 candidate y - L, 8 centre
// y - L).  nr: the slots up to the last nonempty one, which the walk takes in
// order.
struct FlatRuns {
    int rq[6], rq1[6];
    uint32_t fl;
    int nr;
};

__device__ __forceinline__ void flat_runs(const RowGeom &RG, const int32_t *__restrict__ start,
                                          int cb, int ncx, int cx, float fx, float y,
                                          FlatRuns &F) {
    const int ncy = RG.ncy;
    F.fl = 0u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int lo = 0, hi = -1;
        const bool any = column_rows(RG, fx, c - 1, y, lo, hi);
        int ccx = cx + c - 1;
        uint32_t fxs = 0;
        if (ccx < 0) {
            ccx += ncx;
            fxs = 1;
        } else if (ccx >= ncx) {
            ccx -= ncx;
            fxs = 2;
        }
        const int colb = cb + ccx * ncy;
        const bool wlo = lo < 0, whi = hi >= ncy;
        // first segment [ia, ib), second [colb, id)
        int ia = colb + (wlo ? lo + ncy : lo);
        int ib = colb + ((wlo || whi) ? ncy : hi + 1);
        int id = colb + (wlo ? hi + 1 : (whi ? hi - ncy + 1 : 0));
        if (!any) ia = ib = id = colb;
        F.rq[c] = start[ia];
        F.rq1[c] = start[ib];
        F.rq[3 + c] = start[colb];
        F.rq1[3 + c] = start[id];
        F.fl |= (fxs | (wlo ? 4u : 0u)) << (4 * c);
        F.fl |= (fxs | (whi ? 8u : 0u)) << (4 * (3 + c));
    }
    int nr = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) nr = F.rq1[k] > F.rq[k] ? k + 1 : nr;
    F.nr = nr;
}

// NT threads per block, G lanes per agent (in the new cell order): A = NT/G
// agents per block, their sector minima v * A * 4 bytes of dynamic LDS.  G = 1
// suits sparse neighbourhoods (a few dozen candidates); dense ones (hundreds
// to thousands of candidates per agent) share each agent's candidate runs
// among a lane group, which keeps the lanes busy and the LDS per agent small.
// kFov: some env of the launch has a limited field of view.  obs rows hold
// obs_dim floats: the v sectors, then the speed when obs_dim > v.
// kM > 0: full view with v = 8 kM sectors (sector_oct); 0: any v.
//
// kPol (1 mean action, 2 Gaussian sample; not with kTag): the shared policy
// runs on the views the block has just produced, still in LDS, and writes each
// agent's next action (PolFuse).  The views replace the minima in LDS, the
// block's agents are cut into 16-agent tiles spread over its waves, and each
// tile goes through mlp_tile as in the policy kernels.  LDS after the minima:
// the network constants, per-agent speed / env / id, one hidden tile per wave.
// With one lane per agent a wave's agents are its own lanes: each wave runs
// its tiles as soon as its views are written, reading the inputs of its four
// tiles into registers first when they fit one chunk (kc == 1), after which
// its own stretch of the minima (16 rows of 64 words, v >= 16) serves as its
// hidden tile; otherwise (and with four lanes per agent, which needs a block
// barrier) the hidden tiles have a region of their own.  Smaller blocks (lane
// groups of 16 or 64) would read the weights once per tile and are not fused.
struct SweepPolLds {
    int pc, speed, env, id, hid, words;  // offsets in 32-bit words from the minima's start
};
__host__ __device__ constexpr bool sweep_pol_alias(int G, int kc, int vs) {
    return G == 1 && kc == 1 && vs >= 16;
}
__host__ __device__ constexpr SweepPolLds sweep_pol_lds(int min_words, int A, int NT, int G,
                                                        bool alias) {
    const int pc = (min_words + 3) & ~3;
    const int speed = pc + (int)((sizeof(PolConsts) + 15) / 16) * 4;
    const int per_agent = G == 1 ? 0 : A;  // one lane per agent: shuffled from the owner lane
    const int env = speed + per_agent, id = env + per_agent;
    const int hid = (id + per_agent + 3) & ~3;
    return SweepPolLds{pc, speed, env, id, hid, hid + (alias ? 0 : (NT / 64) * 16 * kHidLd / 2)};
}

template <int NT, int G, bool kFov, bool kTag, int kM, int kPol = 0>
__global__ __launch_bounds__(NT) void k_sweep(SortArrays a, const DevEnv *__restrict__ envs,
                                              int n_envs, int Gtot, int v, int obs_dim,
                                              float *__restrict__ obs, float *__restrict__ reward,
                                              int add_ret, PolFuse pf) {
    static_assert(kPol == 0 || !kTag, "the fused policy serves flock envs");
    constexpr int A = NT / G;
    extern __shared__ uint32_t s_min[];  // [channels * v][A] (then the policy's, kPol)
    const int vs = kTag ? 2 * v : v;     // minima per agent
    __shared__ int s_env;
    __shared__ float *s_orow[G == 1 && kPol == 0 ? NT : 1];  // view rows (one lane per agent)
    const int tid = threadIdx.x, slot = tid / G, li = tid % G;
    const int p0 = blockIdx.x * A;
    block_env(&s_env, a.base, n_envs, p0);
    uint32_t *smin = s_min + slot;
    if constexpr (G > 1)
        for (int k = li; k < vs; k += G) smin[k * A] = kInfBits;
    static_assert(kPol == 0 || G <= 4, "the fused policy needs blocks of at least 64 agents");
    const SweepPolLds PL = sweep_pol_lds(vs * A, A, NT, G, sweep_pol_alias(G, pf.kc, vs));
    PolConsts *s_pc = reinterpret_cast<PolConsts *>(s_min + PL.pc);
    float *s_speed = reinterpret_cast<float *>(s_min + PL.speed);
    int *s_pe = reinterpret_cast<int *>(s_min + PL.env);
    int *s_pid = reinterpret_cast<int *>(s_min + PL.id);
    if constexpr (kPol != 0) load_pol_consts(pf.P, s_pc, tid, NT);
    // the strip sort's look-back words and ticket, zero again for the next step
    if (blockIdx.x == 0)
        for (int i = tid; i < a.n_status; i += NT) a.status[i] = 0u;
    __syncthreads();
    const int pos = p0 + slot;
    if constexpr (G == 1 && kPol == 0) {
        if (pos >= Gtot) return;
    }
    // G > 1: every lane reaches the second barrier; a group is active or not as a whole
    const bool active = pos < Gtot;
    int e = s_env;
    if (active)
        while (a.base[e + 1] <= pos) ++e;
    const DevEnv &E = envs[e];
    const int j = pos - E.agent_base;
    float4 me = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int nb = 0, col = 0, ti = 0, my_id = 0;
    if (active) {
        me = load_as<(G > 1)>(E.rec_nxt, j);
        const float2 cs = heading_cs(me.z);
        const float c = cs.x, s = cs.y;
        if constexpr (G == 1)
            for (int k = 0; k < vs; ++k) smin[k * A] = kInfBits;

        const ViewK K{c, s, E.fov_half, E.fov_t, E.sec_scale, (float)v, v};
        ti = kTag ? (load_as<(G > 1)>(E.id_nxt, j) < E.n_chasers ? 1 : 0) : 0;
        const float L = E.box, r2 = E.r2, c2 = E.c2;
        const int ncx = E.ncx, ncy = E.ncy, cb = E.cell_base;
        // one run of candidates [q, q1): template flags say which shifts are nonzero
        auto run = [&](auto sx, auto sy, int q, int q1, float offx, float xi, float offy, float yi,
                       bool minimg) {
            sweep_run<A, G, unroll_for<G>(), kFov, kTag, kM, decltype(sx)::value,
                      decltype(sy)::value>(
                smin, a.sxy, a.stype, ti, q, q1, li, pos, offx, xi, offy, yi, minimg, L, r2, c2, K,
                nb, col);
        };
        using No = std::false_type;
        using Yes = std::true_type;
        if (ncx == 1) {
            run(No{}, No{}, a.start[cb], a.start[cb + 1], 0.0f, me.x, 0.0f, me.y, true);
        } else {
            const int reach = E.reach;
            const int cx = cell_of(me.x, E.inv_cx, ncx);
            const float fx = me.x - (float)cx * E.cw;  // offset within the own column
            const RowGeom RG{E.cw, E.marg, r2, E.inv_cy, ncy};  // held in registers
            // the column's runs over rows [lo, hi]; a column left of column 0
            // wraps to the right edge with its candidates shifted by -L (sx),
            // one right of the last wraps to the left edge with the centre
            // shifted instead; rows wrap likewise
            // the column's runs over rows [lo, hi]; a column left of column 0
            // wraps to the right edge with its candidates shifted by -L (sx),
            // one right of the last wraps to the left edge with the centre
            // shifted instead; rows wrap likewise
            auto column_at = [&](auto sx, int colb, float offx, float xi, int lo, int hi) {
                if (lo < 0) {
                    run(sx, Yes{}, a.start[colb + lo + ncy], a.start[colb + ncy], offx, xi, -L,
                        me.y, false);
                    run(sx, No{}, a.start[colb], a.start[colb + hi + 1], offx, xi, 0.0f, me.y, false);
                } else if (hi >= ncy) {
                    run(sx, No{}, a.start[colb + lo], a.start[colb + ncy], offx, xi, 0.0f, me.y,
                        false);
                    run(sx, No{}, a.start[colb], a.start[colb + hi - ncy + 1], offx, xi, 0.0f,
                        me.y - L, false);
                } else {
                    run(sx, No{}, a.start[colb + lo], a.start[colb + hi + 1], offx, xi, 0.0f, me.y,
                        false);
                }
            };
            // The same from the column's four cell starts st, loaded beforehand.
            auto column = [&](auto sx, float offx, float xi, int lo, int hi, const int (&st)[4]) {
                if (lo < 0) {
                    run(sx, Yes{}, st[0], st[1], offx, xi, -L, me.y, false);
                    run(sx, No{}, st[2], st[3], offx, xi, 0.0f, me.y, false);
                } else if (hi >= ncy) {
                    run(sx, No{}, st[0], st[1], offx, xi, 0.0f, me.y, false);
                    run(sx, No{}, st[2], st[3], offx, xi, 0.0f, me.y - L, false);
                } else {
                    run(sx, No{}, st[0], st[1], offx, xi, 0.0f, me.y, false);
                }
            };
            // Column ox's rows and its starts: the two runs' bounds (the second
            // empty when rows do not wrap); false when no row is within reach.
            // A column left of column 0 wraps to the right edge with its
            // candidates shifted by -L, one right of the last to the left edge
            // with the centre shifted instead.
            auto plan_column = [&](int ox, int &lo, int &hi, int (&st)[4]) {
                const bool any = column_rows(RG, fx, ox, me.y, lo, hi);
                int ccx = cx + ox;
                ccx = ccx < 0 ? ccx + ncx : (ccx >= ncx ? ccx - ncx : ccx);
                const int colb = cb + ccx * ncy;
                int i0 = colb + lo, i1 = colb + hi + 1, i2 = colb, i3 = colb;
                if (lo < 0) {
                    i0 = colb + lo + ncy;
                    i1 = colb + ncy;
                    i3 = colb + hi + 1;
                } else if (hi >= ncy) {
                    i1 = colb + ncy;
                    i3 = colb + hi - ncy + 1;
                }
                if (!any) i0 = i1 = i2 = i3 = colb;
                st[0] = a.start[i0];
                st[1] = a.start[i1];
                st[2] = a.start[i2];
                st[3] = a.start[i3];
                return any;
            };
            if (G == 1 && kFlatRuns && reach == 1) {
                FlatRuns F;
                flat_runs(RG, a.start, cb, ncx, cx, fx, me.y, F);
                // the current run [q, q1) and its shifts; the rest queue in F
                int q = F.rq[0], q1 = F.rq1[0], left = F.nr;
                uint32_t fl = F.fl;
                float offx, xi, offy, yi;
                auto shifts = [&]() {
                    offx = (fl & 1u) ? -L : 0.0f;
                    xi = (fl & 2u) ? me.x - L : me.x;
                    offy = (fl & 4u) ? -L : 0.0f;
                    yi = (fl & 8u) ? me.y - L : me.y;
                };
                shifts();
                // kFlatUnroll candidates per step, those past the run's end
                // masked (the position arrays are padded for the reads); each
                // step loads the next one's before its tests: the rest of this
                // run, else the next queued run's start (a stale but in-range
                // start once none is left)
                float2 pj[kFlatUnroll];
#pragma unroll
                for (int u = 0; u < kFlatUnroll; ++u) pj[u] = a.sxy[q + u];
                while (true) {
                    const int qn = q + kFlatUnroll < q1 ? q + kFlatUnroll : F.rq[1];
                    float2 pn[kFlatUnroll];
#pragma unroll
                    for (int u = 0; u < kFlatUnroll; ++u) pn[u] = a.sxy[qn + u];
                    const int rem = q1 - q, so = pos - q;  // slots in the run; the agent's own
                    // most runs have no candidate-side shift: a step in which no
                    // lane of the wave has one leaves out the two additions
                    if (__any((fl & 5u) != 0u)) {
#pragma unroll
                        for (int u = 0; u < kFlatUnroll; ++u)
                            test_pair<A, kFov, kTag, kM, true, true>(
                                smin, a.stype, ti, pj[u], q + u, u < rem && u != so, offx, xi,
                                offy, yi, false, L, r2, c2, K, nb, col);
                    } else {
#pragma unroll
                        for (int u = 0; u < kFlatUnroll; ++u)
                            test_pair<A, kFov, kTag, kM, false, false>(
                                smin, a.stype, ti, pj[u], q + u, u < rem && u != so, offx, xi,
                                offy, yi, false, L, r2, c2, K, nb, col);
                    }
                    q += kFlatUnroll;
                    if (q >= q1) {
                        // next slot (an empty one costs a step of masked tests)
                        if (--left <= 0) break;
#pragma unroll
                        for (int k = 0; k < 5; ++k) {
                            F.rq[k] = F.rq[k + 1];
                            F.rq1[k] = F.rq1[k + 1];
                        }
                        fl >>= 4;
                        q = F.rq[0];
                        q1 = F.rq1[0];
                        shifts();
                    }
#pragma unroll
                    for (int u = 0; u < kFlatUnroll; ++u) pj[u] = pn[u];
                }
            } else if constexpr (kFov || kTag || kPol != 0) {
                // (the limited-view and tag sweeps, whose runs are long: loading
                // the next column's starts ahead measured no faster there, 56.0
                // against 56.5 us per step of 16,000 agents at 128 sectors and
                // 64 lanes, and takes 6 to 7 more registers, as it would in the
                // policy sweeps, which already hold more than 64)
                for (int ox = -reach; ox <= reach; ++ox) {
                    int lo, hi;
                    if (!column_rows(RG, fx, ox, me.y, lo, hi)) continue;
                    const int ccx = cx + ox;
                    if (ccx < 0) column_at(Yes{}, cb + (ccx + ncx) * ncy, -L, me.x, lo, hi);
                    else if (ccx >= ncx) column_at(No{}, cb + (ccx - ncx) * ncy, 0.0f, me.x - L, lo, hi);
                    else column_at(No{}, cb + ccx * ncy, 0.0f, me.x, lo, hi);
                }
            } else {
                // each column's starts are loaded while the column before it
                // is swept, so a lane group does not wait for them between runs
                // (4 lanes, 20 x 50,000 clustered agents: 151 -> 143 us per
                // step; 16 lanes, uniform: 291 -> 268)
                int lo = 0, hi = -1, st[4];
                bool any = plan_column(-reach, lo, hi, st);
                for (int ox = -reach; ox <= reach; ++ox) {
                    int nlo = 0, nhi = -1, nst[4] = {0, 0, 0, 0};
                    const bool nany = ox < reach && plan_column(ox + 1, nlo, nhi, nst);
                    if (any) {
                        const int ccx = cx + ox;
                        if (ccx < 0) column(Yes{}, -L, me.x, lo, hi, st);
                        else if (ccx >= ncx) column(No{}, 0.0f, me.x - L, lo, hi, st);
                        else column(No{}, 0.0f, me.x, lo, hi, st);
                    }
                    any = nany;
                    lo = nlo;
                    hi = nhi;
#pragma unroll
                    for (int k = 0; k < 4; ++k) st[k] = nst[k];
                }
            }
        }
    }  // active

    if constexpr (G > 1) {
        __syncthreads();  // the group's minima are complete
        if (kPol == 0 && !active) return;
#pragma unroll
        for (int m = G / 2; m >= 1; m >>= 1) {
            nb += __shfl_xor(nb, m, 64);
            col += __shfl_xor(col, m, 64);
        }
    }
    constexpr bool kGl = G > 1;
    // A view value from a sector minimum; with kPol it also replaces the minimum in LDS.
    auto view = [&](int k, float inv_r) {
        const uint32_t m = smin[k * A];
        const float o = m == kInfBits ? 0.0f : 1.0f - __builtin_amdgcn_sqrtf(__uint_as_float(m)) * inv_r;
        if constexpr (kPol != 0) smin[k * A] = __float_as_uint(o);
        return o;
    };
    // One lane per agent: rows of 4, 8, 16, 32 or 64 views (no speed column)
    // leave the wave whole, vs / 4 lanes to a row, so that each store instruction writes
    // 64 / (vs / 4) whole rows rather than 16 bytes of each of 64 rows.
    const bool rows_whole =
        G == 1 && kPol == 0 && obs_dim == vs && vs >= 4 && vs <= 64 && (vs & (vs - 1)) == 0;
    if (active) {
        // agent-order rows are addressed by id: an id out of range (a sort
        // that went wrong) writes agent 0's rows instead of outside them
        const int id0 = load_as<kGl>(E.id_nxt, j);
        const int id = (unsigned)id0 < (unsigned)E.n ? id0 : 0;
        my_id = id;
        const float inv_r = E.inv_radius;
        float *orow = obs ? obs + ((size_t)E.agent_base + id) * obs_dim : E.obs + (size_t)id * obs_dim;
        if (li == 0 && obs_dim > vs) store_as<kGl>(orow, vs, me.w);  // speed after the move (Sec. 4.1)
        if constexpr (G > 1) {
            for (int k = li; k < vs; k += G) store_as<kGl>(orow, k, view(k, inv_r));
        } else if (rows_whole) {
            // the views in place of the minima, the row's address beside them
            for (int k = 0; k < vs; ++k) smin[k * A] = __float_as_uint(view(k, inv_r));
            if constexpr (kPol == 0) s_orow[slot] = orow;
        } else if ((obs_dim & 3) == 0 && (vs & 3) == 0) {
            for (int k = 0; k < vs; k += 4) {
                float o[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) o[u] = view(k + u, inv_r);
                *reinterpret_cast<float4 *>(orow + k) = make_float4(o[0], o[1], o[2], o[3]);
            }
        } else {
            for (int k = 0; k < vs; ++k) orow[k] = view(k, inv_r);
        }
        if (li == 0) {
            const float r =
                (kTag && ti) ? E.r_catch * (float)col : E.r_nb * (float)nb + E.r_col * (float)col;
            if (reward) reward[E.agent_base + id] = r;
            else if (E.rew) store_as<kGl>(E.rew, id, r);
            if (add_ret) store_as<kGl>(E.ret_nxt, j, load_as<kGl>(E.ret_nxt, j) + (double)r);
            if (E.nb) {
                store_as<kGl>(E.nb, id, nb);
                store_as<kGl>(E.col, id, col);
            }
            if constexpr (kPol != 0 && G > 1) {
                s_speed[slot] = me.w;
                s_pe[slot] = e;
                s_pid[slot] = id;
            }
        }
    } else if constexpr (kPol != 0 && G > 1) {
        if (li == 0) s_pe[slot] = -1;
    }
    if constexpr (G == 1 && kPol == 0) {
        if (rows_whole) {
            // The lanes left here are the wave's active ones, a prefix of it
            // (in the last wave of a launch the others have returned): they
            // share out the n_act rows' vs / 4 pieces, piece t = row t / lpr,
            // columns 4 (t % lpr) on.
            wave_lds_fence();
            const int lane = tid & 63, w0 = tid - lane;
            const int n_act = __popcll(__ballot(1));
            const int lpr = vs >> 2, lg = __builtin_ctz(lpr);
            for (int t = lane; t < n_act * lpr; t += n_act) {
                const int r = t >> lg, c4 = 4 * (t & (lpr - 1));
                const uint32_t *col4 = s_min + c4 * A + w0 + r;
                *reinterpret_cast<float4 *>(s_orow[w0 + r] + c4) =
                    make_float4(__uint_as_float(col4[0]), __uint_as_float(col4[A]),
                                __uint_as_float(col4[2 * A]), __uint_as_float(col4[3 * A]));
            }
        }
    }
    // The policy's action of a tile's agent from its output pre-activations
    // (lanes g == 0 of a valid column write).
    auto write_act = [&](float2 z, int pe, int idj, bool wr) {
        if (!wr) return;
        const DevEnv &Ej = envs[pe];
        const int64_t row = (int64_t)Ej.agent_base + idj;
        const float2 ev = kPol == 2 ? pf.eps[row] : make_float2(0.0f, 0.0f);
        const float2 av = pol_output<kPol == 2>(z, pf.max_turn, pf.max_dspeed, ev, pf.sig0, pf.sig1,
                                                pf.logp_c,
                                                (kPol == 2 && pf.logp) ? pf.logp + row : nullptr);
        if (pf.act) pf.act[row] = av;
        else reinterpret_cast<float2 *>(Ej.act)[idj] = av;
    };
    // weight fragments read at use from global memory (cached): held in
    // registers they would lower the whole kernel's occupancy, staged in LDS
    // they made the policy phase LDS-bound (measured slower)
    const int lane = tid & 63, g = lane >> 4, colx = lane & 15;
    auto w1a = [&](int c, int t) { return pf.P.w1[(c * 4 + t) * 64 + lane]; };
    auto w2a = [&](int c, int t) { return pf.P.w2[(c * 4 + t) * 64 + lane]; };
    auto w3a = [&](int c) { return pf.P.w3[c * 64 + lane]; };
    if constexpr (kPol != 0 && G == 1) {
        const int w0 = tid - lane;  // the wave's first slot
        const int my_e = active ? e : -1;
        const float my_sp = me.w;
        wave_lds_fence();           // the wave's views in LDS before its reads
        // inputs of tile t (agents w0 + 16 t + col, owned by lane 16 t + col):
        // the view, then the speed when the row carries it, zero beyond
        auto input = [&](int t, int k, int pe, float sp) {
            float o = 0.0f;
            if (pe >= 0) {
                if (k < vs) o = __uint_as_float(s_min[k * A + w0 + 16 * t + colx]);
                else if (k == vs && obs_dim > vs) o = sp;
            }
            return (__bf16)o;
        };
        if (sweep_pol_alias(G, pf.kc, vs)) {
            bf16x8 xr[4];
            int te[4], ti4[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int src = 16 * t + colx;
                te[t] = __shfl(my_e, src, 64);
                ti4[t] = __shfl(my_id, src, 64);
                const float sp = __shfl(my_sp, src, 64);
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) xr[t][jj] = input(t, 8 * g + jj, te[t], sp);
            }
            wave_lds_fence();  // every lane's reads before the stretch becomes the hidden tile
            // row r: minima row r of the wave's stretch, skewed by (r % 8) * 4 words
            auto hrow = [&](int r) {
                return reinterpret_cast<__bf16 *>(s_min + r * A + w0 + (r & 7) * 4);
            };
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float2 z =
                    mlp_tile(1, [&](int) { return xr[t]; }, w1a, w2a, w3a, *s_pc, hrow, lane);
                write_act(z, te[t], ti4[t], g == 0 && te[t] >= 0);
            }
        } else {
            __bf16 *s_hid = reinterpret_cast<__bf16 *>(s_min + PL.hid) + (size_t)(tid >> 6) * 16 * kHidLd;
            auto hrow = [&](int r) { return s_hid + r * kHidLd; };
            for (int t = 0; t < 4; ++t) {
                const int src = 16 * t + colx;
                const int pe = __shfl(my_e, src, 64), idj = __shfl(my_id, src, 64);
                const float sp = __shfl(my_sp, src, 64);
                auto xb = [&](int c) {
                    bf16x8 x;
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) x[jj] = input(t, 32 * c + 8 * g + jj, pe, sp);
                    return x;
                };
                const float2 z = mlp_tile(pf.kc, xb, w1a, w2a, w3a, *s_pc, hrow, lane);
                write_act(z, pe, idj, g == 0 && pe >= 0);
            }
        }
        return;
    }
    if constexpr (kPol != 0) {
        __syncthreads();  // every agent's view, speed and row are in LDS
        constexpr int kTiles = (A + 15) / 16;
        const int wid = tid >> 6;
        __bf16 *s_hid = reinterpret_cast<__bf16 *>(s_min + PL.hid) + (size_t)wid * 16 * kHidLd;
        auto hrow = [&](int r) { return s_hid + r * kHidLd; };
        if (wid >= kTiles) return;
        for (int tile = wid; tile < kTiles; tile += NT / 64) {
            const int sl = tile * 16 + colx;
            const int pe = sl < A ? s_pe[sl] : -1;
            const bool valid = pe >= 0;
            // inputs 32 c + 8 g .. + 7 of agent sl: the view, then the speed when
            // the row carries it, zero beyond
            auto xb = [&](int c) {
                bf16x8 x;
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const int k = 32 * c + 8 * g + jj;
                    float o = 0.0f;
                    if (valid) {
                        if (k < vs) o = __uint_as_float(s_min[k * A + sl]);
                        else if (k == vs && obs_dim > vs) o = s_speed[sl];
                    }
                    x[jj] = (__bf16)o;
                }
                return x;
            };
            const float2 z = mlp_tile(pf.kc, xb, w1a, w2a, w3a, *s_pc, hrow, lane);
            write_act(z, pe, valid ? s_pid[sl] : 0, g == 0 && valid);
        }
    }
}

// ------------------------------------------------------------------ helpers

__global__ void k_clear(int32_t *count, int64_t C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C) count[i] = 0;
}

__global__ void k_load_state(const float *x, const float *y, const float *th, const float *sp,
                             float4 *rec, int32_t *id, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rec[i] = make_float4(x[i], y[i], th[i], sp[i]);
    id[i] = i;
}

__global__ void k_store_state(const float4 *rec, const int32_t *id, float *x, float *y, float *th,
                              float *sp, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float4 r = rec[p];
    const int i = id[p];
    x[i] = r.x;
    y[i] = r.y;
    th[i] = r.z;
    sp[i] = r.w;
}

__global__ void k_store_returns(const double *ret, const int32_t *id, double *out, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) out[id[p]] = ret[p];
}

__global__ void k_load_returns(const double *in, const int32_t *id, double *ret, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) ret[p] = in[id[p]];
}

__global__ void k_zero_f64(double *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_copy_i32(const int32_t *src, int32_t *dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

int env_sort_recs_for(int n_envs, int64_t max_env_agents, int64_t max_env_cells) {
    if (n_envs < 64 || max_env_cells > 16384) return 0;
    // (envs up to 16,384 agents: a 20,000-agent env in a batch of smaller
    // ones keeps its block busy long after the rest are done)
    for (int r = 2; r <= 16; r *= 2)
        if (max_env_agents <= (int64_t)r * kEnvNT) return r;
    return 0;
}

int scan_blocks_for(int64_t C, int64_t max_env_cells) {
    return max_env_cells <= kScanTile ? 0 : (int)((C + kTile2 - 1) / kTile2);
}

void carve_sort(Carver &cv, int64_t G, int64_t C, int E, SortArrays *a, int64_t S) {
    const int64_t nb = (C + kTile2 - 1) / kTile2;  // partials of the two-level scan
    a->key = cv.take<int32_t>(G);
    a->slot = cv.take<int32_t>(G);
    a->tmp = cv.take<float4>(G);
    a->sxy = cv.take<float2>(G + kSortPad);
    a->stype = cv.take<uint8_t>(G + kSortPad);
    a->count = cv.take<int32_t>(C);
    a->start = cv.take<int32_t>(C + 1);
    a->part = cv.take<int32_t>(nb + 1);
    a->envs[0] = cv.take<DevEnv>(E);
    a->envs[1] = cv.take<DevEnv>(E);
    a->base = cv.take<int32_t>(E + 1);
    a->strip_env = S > 0 ? cv.take<int32_t>(S) : nullptr;
    a->status = S > 0 ? cv.take<uint32_t>(S + 1) : nullptr;
    a->n_status = S > 0 ? (int32_t)(S + 1) : 0;
}

bool strips_allowed(const DevEnv &d) {
    // at most one column per step (half a column leaves room for the rounding
    // of the column boundaries), and one column's cells fit the block
    return d.ncy <= kStripCells && d.s_max <= 0.5f * d.cw;
}

int strip_cols_for(const DevEnv &d, int64_t G) {
    // about G / 512 agents per strip (at least 512, at most 4,096), so a
    // large batch gives hundreds of blocks and a small one still several
    const double target = std::min(4096.0, std::max(512.0, (double)G / 512.0));
    const double per_col = (double)std::max(d.n, 1) / d.ncx;
    int cols = (int)std::lround(target / per_col);
    cols = std::max(1, std::min(cols, kStripCells / d.ncy));
    return std::min(cols, d.ncx);
}

// LDS of a strip block: cells, then 16 bytes per listed agent.
static size_t strip_lds_bytes(int cells, int cap) {
    return ((size_t)((cells + 3) & ~3) + 4 * (size_t)cap) * sizeof(int);
}

void plan_strip_launch(StepPlan *p, const DevEnv *envs, int n_envs) {
    int cells = 1;
    double own = 1.0;
    for (int e = 0; e < n_envs; ++e) {
        const DevEnv &d = envs[e];
        cells = std::max(cells, d.strip_cols * d.ncy);
        own = std::max(own, (double)std::max(d.n, 1) / d.ncx * d.strip_cols);
    }
    // half again the largest expected strip (uniform density), within 64 KiB
    const int fit = (int)((65536 / sizeof(int) - ((cells + 3) & ~3)) / 4);
    p->strip_cells = cells;
    p->strip_cap = std::max(0, std::min((int)std::ceil(1.5 * own), fit));
}

// Whether every block of the plan's strip sort is resident at once (as the
// runtime's occupancy calculation for this kernel and LDS size says), so the
// block index can serve as the strip: a strip then only ever waits for
// strips that are running.  The CU count is read once per device.
static int strip_direct(const StepPlan &p) {
    static int cus_of[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cus_of[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            return 0;
        cus_of[dev] = cus;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(k_strip_sort<kStripNT>), kStripNT,
            strip_lds_bytes(p.strip_cells, p.strip_cap)) != hipSuccess)
        return 0;
    // the padded grid (a multiple of kXcds blocks) must be resident too
    const int64_t blocks = (p.strips + kXcds - 1) / kXcds * kXcds;
    return blocks <= (int64_t)cus_of[dev] * per_cu ? 1 : 0;
}

int64_t assign_strips(DevEnv *const *tabs, int n_tabs, int n_envs, int64_t G,
                      std::vector<int32_t> *strip_env) {
    int64_t S = 0;
    if (strip_env) strip_env->clear();
    for (int e = 0; e < n_envs; ++e) {
        const int cols = strip_cols_for(tabs[0][e], G);
        const int ns = (tabs[0][e].ncx + cols - 1) / cols;
        for (int k = 0; k < n_tabs; ++k) {
            tabs[k][e].strip_base = (int32_t)S;
            tabs[k][e].strip_cols = cols;
            tabs[k][e].n_strips = ns;
        }
        if (strip_env) strip_env->insert(strip_env->end(), ns, e);
        S += ns;
    }
    return S;
}

// Descriptor tables and agent offsets of a one-env plan, written from the
// kernel's by-value arguments (no copy from host memory), and the plan's cell
// counts zeroed: what a step needs in its sort scratch before it starts.
__global__ void k_bind_one(SortArrays a, DevEnv d0, DevEnv d1, int32_t n, int64_t C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < C) a.count[i] = 0;
    if (i < a.n_status) a.status[i] = 0u;
    if (i == 0) {
        a.envs[0][0] = d0;
        a.envs[1][0] = d1;
        a.base[0] = 0;
        a.base[1] = n;
    }
}

hipError_t launch_bind_one(const StepPlan &p, const DevEnv &d0, const DevEnv &d1, int32_t n,
                           hipStream_t s) {
    const int64_t c = std::max<int64_t>(std::max<int64_t>(p.C, p.a.n_status), 1);
    hipLaunchKernelGGL(k_bind_one, dim3(blocks_for(c, 256)), dim3(256), 0, s, p.a, d0, d1, n, p.C);
    return hipGetLastError();
}

bool plan_fuses_policy(const StepPlan &p) { return !p.tag && (p.lanes == 1 || p.lanes == 4); }

hipError_t launch_clear(const StepPlan &p, hipStream_t s) {
    const int64_t n = p.C > 0 ? p.C : 1;
    hipLaunchKernelGGL(k_clear, dim3(blocks_for(n, 256)), dim3(256), 0, s, p.a.count, p.C);
    if (p.a.n_status > 0)
        hipLaunchKernelGGL(k_clear, dim3(blocks_for(p.a.n_status, 256)), dim3(256), 0, s,
                           reinterpret_cast<int32_t *>(p.a.status), (int64_t)p.a.n_status);
    return hipGetLastError();
}

namespace {
template <int NT, int G, bool kFov, bool kTag, int kM = 0, int kPol = 0>
void launch_sweep_v(const StepPlan &p, const DevEnv *envs, int Gtot, float *obs, float *reward,
                    int add_return, hipStream_t s, const PolFuse *pf) {
    constexpr int A = NT / G;
    const int vs = (kTag ? 2 : 1) * p.v, min_words = vs * A;
    const size_t lds =
        (size_t)(kPol ? sweep_pol_lds(min_words, A, NT, G, sweep_pol_alias(G, pf->kc, vs)).words
                      : min_words) *
        sizeof(uint32_t);
    hipLaunchKernelGGL((k_sweep<NT, G, kFov, kTag, kM, kPol>), dim3(blocks_for(Gtot, A)), dim3(NT),
                       lds, s, p.a, envs, p.n_envs, Gtot, p.v, p.obs_dim, obs, reward, add_return,
                       pf ? *pf : PolFuse{});
}

// Flock plans: the view variant (limited view, or 8 / 16 / 32 sectors without
// the arctangent) and, with pf, the fused policy's output mode.
template <int NT, int G, int kPol>
void launch_sweep_flock(const StepPlan &p, const DevEnv *envs, int Gtot, float *obs, float *reward,
                        int add_return, hipStream_t s, const PolFuse *pf) {
    if (p.fov) launch_sweep_v<NT, G, true, false, 0, kPol>(p, envs, Gtot, obs, reward, add_return, s, pf);
    else if (p.v == 8) launch_sweep_v<NT, G, false, false, 1, kPol>(p, envs, Gtot, obs, reward, add_return, s, pf);
    else if (p.v == 16) launch_sweep_v<NT, G, false, false, 2, kPol>(p, envs, Gtot, obs, reward, add_return, s, pf);
    else if (p.v == 32) launch_sweep_v<NT, G, false, false, 4, kPol>(p, envs, Gtot, obs, reward, add_return, s, pf);
    else launch_sweep_v<NT, G, false, false, 0, kPol>(p, envs, Gtot, obs, reward, add_return, s, pf);
}

template <int NT, int G>
void launch_sweep(const StepPlan &p, const DevEnv *envs, int Gtot, float *obs, float *reward,
                  int add_return, hipStream_t s, const PolFuse *pf) {
    if (p.tag) {
        if (p.fov) launch_sweep_v<NT, G, true, true>(p, envs, Gtot, obs, reward, add_return, s, nullptr);
        else launch_sweep_v<NT, G, false, true>(p, envs, Gtot, obs, reward, add_return, s, nullptr);
    } else if (!pf) {
        launch_sweep_flock<NT, G, 0>(p, envs, Gtot, obs, reward, add_return, s, nullptr);
    } else if constexpr (G <= 4) {
        if (pf->mode == 2) launch_sweep_flock<NT, G, 2>(p, envs, Gtot, obs, reward, add_return, s, pf);
        else launch_sweep_flock<NT, G, 1>(p, envs, Gtot, obs, reward, add_return, s, pf);
    }
}
}  // namespace

hipError_t launch_phase(const StepPlan &p, int table, StepPhase phase, int do_move,
                        const float *act, float *obs, float *reward, int add_return,
                        hipStream_t s, const PolFuse *pf, float *act_copy) {
    if (pf && !plan_fuses_policy(p)) return hipErrorInvalidValue;
    if (p.G == 0) return hipSuccess;
    const int G = (int)p.G, C = (int)p.C;
    const DevEnv *envs = p.a.envs[table & 1];
    const unsigned nb = blocks_for(G, kBlock);
    switch (phase) {
        case kPhaseMove:
            if (p.env_sort_recs == 0 && p.strips > 0 && p.strip_now) {
                // direct: strips per XCD (blocks = kXcds x that, the last few idle)
                const int per_xcd = strip_direct(p) ? (int)((p.strips + kXcds - 1) / kXcds) : 0;
                const unsigned nblk = per_xcd ? (unsigned)(per_xcd * kXcds) : (unsigned)p.strips;
                hipLaunchKernelGGL(k_strip_sort<kStripNT>, dim3(nblk), dim3(kStripNT),
                                   strip_lds_bytes(p.strip_cells, p.strip_cap), s, p.a, envs,
                                   p.n_envs, C, G, (int)p.strips, do_move,
                                   reinterpret_cast<const float2 *>(act), p.tag,
                                   reinterpret_cast<float2 *>(act_copy), p.strip_cap, per_xcd,
                                   p.strip_wait);
                break;
            }
            if (p.env_sort_recs > 0) {
                const size_t lds = (size_t)p.max_env_cells * sizeof(int);
                const float2 *a2 = reinterpret_cast<const float2 *>(act);
                float2 *ac2 = reinterpret_cast<float2 *>(act_copy);
                const dim3 grid(p.n_envs), block(kEnvNT);
                switch (p.env_sort_recs) {
                    case 2: hipLaunchKernelGGL(k_env_sort<2>, grid, block, lds, s, p.a, envs, p.n_envs, C, do_move, a2, p.tag, ac2); break;
                    case 4: hipLaunchKernelGGL(k_env_sort<4>, grid, block, lds, s, p.a, envs, p.n_envs, C, do_move, a2, p.tag, ac2); break;
                    case 8: hipLaunchKernelGGL(k_env_sort<8>, grid, block, lds, s, p.a, envs, p.n_envs, C, do_move, a2, p.tag, ac2); break;
                    default: hipLaunchKernelGGL(k_env_sort<16>, grid, block, lds, s, p.a, envs, p.n_envs, C, do_move, a2, p.tag, ac2); break;
                }
                break;
            }
            hipLaunchKernelGGL(k_move_count, dim3(blocks_for(G, kBlock * kMoveRecs)), dim3(kBlock),
                               0, s, p.a, envs, p.n_envs, G, do_move,
                               reinterpret_cast<const float2 *>(act),
                               reinterpret_cast<float2 *>(act_copy));
            break;
        case kPhaseScan:
            if (p.env_sort_recs > 0 || (p.strips > 0 && p.strip_now)) break;  // one-kernel sorts
            if (p.scan_blocks == 0) {
                if (p.max_env_cells <= 2048)
                    hipLaunchKernelGGL((k_scan_env<256, 8>), dim3(p.n_envs), dim3(256), 0, s,
                                       p.a.count, p.a.start, envs, p.n_envs, C);
                else
                    hipLaunchKernelGGL((k_scan_env<kScanNT, kScanItems>), dim3(p.n_envs),
                                       dim3(kScanNT), 0, s, p.a.count, p.a.start, envs, p.n_envs, C);
            } else {
                hipLaunchKernelGGL(k_tile_sums, dim3(p.scan_blocks), dim3(kScan2NT), 0, s,
                                   p.a.count, p.a.part, C);
                if (p.scan_blocks <= kDirectTiles) {
                    hipLaunchKernelGGL(k_scan_down<true>, dim3(p.scan_blocks), dim3(kScan2NT), 0,
                                       s, p.a.count, p.a.part, p.a.start, C);
                } else {
                    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kScan2NT), 0, s, p.a.part,
                                       p.scan_blocks);
                    hipLaunchKernelGGL(k_scan_down<false>, dim3(p.scan_blocks), dim3(kScan2NT), 0,
                                       s, p.a.count, p.a.part, p.a.start, C);
                }
            }
            break;
        case kPhaseScatter:
            if (p.env_sort_recs > 0 || (p.strips > 0 && p.strip_now)) break;  // one-kernel sorts
            hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, s, p.a, envs, p.n_envs, G,
                               p.tag);
            break;
        case kPhaseSweep: {
            const int lanes = p.lanes;
            if (lanes == 4) launch_sweep<256, 4>(p, envs, G, obs, reward, add_return, s, pf);
            else if (lanes == 16) launch_sweep<256, 16>(p, envs, G, obs, reward, add_return, s, pf);
            else if (lanes == 64) launch_sweep<256, 64>(p, envs, G, obs, reward, add_return, s, pf);
            else if ((p.tag ? 2 * p.v : p.v) <= 32)
                launch_sweep<256, 1>(p, envs, G, obs, reward, add_return, s, pf);
            else launch_sweep<64, 1>(p, envs, G, obs, reward, add_return, s, pf);
            break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_step(const StepPlan &p, int table, int do_move, const float *act, float *obs,
                       float *reward, int add_return, hipStream_t s, hipEvent_t *ev,
                       const PolFuse *pf, float *act_copy) {
    if (p.G == 0) return hipSuccess;
    const StepPhase order[4] = {kPhaseMove, kPhaseScan, kPhaseScatter, kPhaseSweep};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
        if (ev) (void)hipEventRecord(ev[k], s);
        e = launch_phase(p, table, order[k], do_move, act, obs, reward, add_return, s, pf,
                         act_copy);
    }
    if (ev) (void)hipEventRecord(ev[4], s);
    return e;
}

hipError_t launch_load_state(const float *x, const float *y, const float *th, const float *sp,
                             float4 *rec, int32_t *id, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_state, dim3(blocks_for(n, 256)), dim3(256), 0, s, x, y, th, sp, rec,
                       id, n);
    return hipGetLastError();
}

hipError_t launch_store_state(const float4 *rec, const int32_t *id, float *x, float *y, float *th,
                              float *sp, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_state, dim3(blocks_for(n, 256)), dim3(256), 0, s, rec, id, x, y, th,
                       sp, n);
    return hipGetLastError();
}

hipError_t launch_store_returns(const double *ret, const int32_t *id, double *out, int n,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_store_returns, dim3(blocks_for(n, 256)), dim3(256), 0, s, ret, id, out, n);
    return hipGetLastError();
}

hipError_t launch_load_returns(const double *in, const int32_t *id, double *ret, int n,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_returns, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, id, ret, n);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace flock
