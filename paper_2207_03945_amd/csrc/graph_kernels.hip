// graph_kernels.hip -- the graph interaction: opinion dynamics over CSR edges.
//
// Sec. 2.1 of arXiv:2207.03945 gives interactions over the edges of a graph
// as the engine's second base pattern, with an opinion model as example:
// for each edge (me, you) of weight w_e, when |op_me - op_you| < threshold,
// me's new opinion moves toward you's current opinion,
//     new <- (1 - s w_e) new + s w_e op_you        (s = strength),
// starting from new = op_me; a self interaction then commits the new
// opinions.  A step reads op_in and writes op_out (the caller ping-pongs).
//
// Each node applies its incoming edges in CSR order, so its new opinion is
// the composition of per-edge affine maps x -> (1 - w) x + w y.  G lanes share
// a node: lane l applies the edges of the l-th contiguous chunk of the row to
// an affine map (a, b), the G maps are composed in chunk order by a shuffle
// butterfly, and lane 0 applies the result to op_me.  With G = 1 the lane
// runs the recurrence itself, in exactly the order the model states.
// Arithmetic: the threshold test in FP32 on the FP32 opinions, the updates
// in FP64, one rounding to FP32 at the end.
//
// Memory safety: row ranges are clamped to [0, n_edges] and edges whose
// `you` lies outside [0, n) are skipped, whatever the arrays hold.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "flock_internal.h"

namespace flock {

namespace {

constexpr int kGraphBlock = 256;
// Edges a lane loads at once: their targets, weights and then the targets'
// opinions are each one round of loads in flight, instead of two dependent
// loads per edge (rows of power-law graphs reach thousands of edges, and a
// lane's chain of loads over its chunk sets the step's critical path).
// MI355X, 1M nodes, mean degree 14, 16 lanes: 0.208 ms per step one edge at
// a time, 0.139 with 4, 0.148 with 8, 0.217 with 16 (short chunks then load
// mostly padding).
constexpr int kEdgeBatch = 4;

// Loads of edges e .. e + kEdgeBatch - 1 of [e, c1) (e < c1): slots past c1
// read edge c1 - 1 and targets outside [0, n) read node 0; ok[u] says which
// slots hold an edge to apply.
__device__ __forceinline__ void load_edges(int64_t e, int64_t c1, int64_t n,
                                           const int32_t *__restrict__ col,
                                           const float *__restrict__ weight,
                                           const float *__restrict__ op_in, bool (&ok)[kEdgeBatch],
                                           float (&wt)[kEdgeBatch], float (&you)[kEdgeBatch]) {
    int32_t j[kEdgeBatch];
#pragma unroll
    for (int u = 0; u < kEdgeBatch; ++u) {
        const int64_t k = e + u < c1 ? e + u : c1 - 1;
        j[u] = col[k];
        wt[u] = weight[k];
        ok[u] = e + u < c1 && j[u] >= 0 && (int64_t)j[u] < n;
    }
#pragma unroll
    for (int u = 0; u < kEdgeBatch; ++u) you[u] = op_in[ok[u] ? j[u] : 0];
}

template <int G>
__global__ __launch_bounds__(kGraphBlock) void k_opinion(int64_t n, int64_t n_edges,
                                                         const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const float *__restrict__ weight,
                                                         float thr, double strength,
                                                         const float *__restrict__ op_in,
                                                         float *__restrict__ op_out) {
    constexpr int A = kGraphBlock / G;  // nodes per block
    const int tid = threadIdx.x, slot = tid / G, li = tid % G;
    const int64_t i = (int64_t)blockIdx.x * A + slot;
    const bool active = i < n;
    float me = 0.0f;
    int64_t e0 = 0, e1 = 0;
    if (active) {
        me = op_in[i];
        e0 = row_ptr[i];
        e1 = row_ptr[i + 1];
        e0 = e0 < 0 ? 0 : (e0 > n_edges ? n_edges : e0);
        e1 = e1 < e0 ? e0 : (e1 > n_edges ? n_edges : e1);
    }
    if constexpr (G == 1) {
        if (!active) return;
        double x = (double)me;
        for (int64_t e = e0; e < e1; e += kEdgeBatch) {
            bool ok[kEdgeBatch];
            float wt[kEdgeBatch], you[kEdgeBatch];
            load_edges(e, e1, n, col, weight, op_in, ok, wt, you);
#pragma unroll
            for (int u = 0; u < kEdgeBatch; ++u) {  // in edge order
                if (ok[u] && fabsf(me - you[u]) < thr) {
                    const double w = strength * (double)wt[u];
                    x = (1.0 - w) * x + w * (double)you[u];
                }
            }
        }
        op_out[i] = (float)x;
    } else {
        const int64_t len = e1 - e0;
        const int64_t chunk = (len + G - 1) / G;
        int64_t c0 = e0 + (int64_t)li * chunk;
        c0 = c0 < e1 ? c0 : e1;
        const int64_t c1 = c0 + chunk < e1 ? c0 + chunk : e1;
        double a = 1.0, b = 0.0;  // x -> a x + b over this lane's chunk
        for (int64_t e = c0; e < c1; e += kEdgeBatch) {
            bool ok[kEdgeBatch];
            float wt[kEdgeBatch], you[kEdgeBatch];
            load_edges(e, c1, n, col, weight, op_in, ok, wt, you);
#pragma unroll
            for (int u = 0; u < kEdgeBatch; ++u) {  // in edge order
                if (ok[u] && fabsf(me - you[u]) < thr) {
                    const double w = strength * (double)wt[u];
                    a = (1.0 - w) * a;
                    b = (1.0 - w) * b + w * (double)you[u];
                }
            }
        }
        // butterfly: after level `off`, each lane holds the composition of
        // the 2 off consecutive chunks round it, later chunks applied last
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            const double pa = __shfl_xor(a, off, 64);
            const double pb = __shfl_xor(b, off, 64);
            if (li & off) {  // mine is the later range
                b = a * pb + b;
                a = a * pa;
            } else {
                b = pa * b + pb;
                a = pa * a;
            }
        }
        if (active && li == 0) op_out[i] = (float)(a * (double)me + b);
    }
}

template <int G>
void launch_opinion(int64_t n, int64_t n_edges, const int64_t *row_ptr, const int32_t *col,
                    const float *weight, float thr, double strength, const float *op_in,
                    float *op_out, hipStream_t s) {
    constexpr int A = kGraphBlock / G;
    const int64_t blocks = (n + A - 1) / A;
    hipLaunchKernelGGL(k_opinion<G>, dim3((unsigned)blocks), dim3(kGraphBlock), 0, s, n, n_edges,
                       row_ptr, col, weight, thr, strength, op_in, op_out);
}

// Lanes per node from the mean degree.  Power-law rows are uneven, so wide
// groups pay off early: on MI355X a 1M-node graph of mean degree 14 steps in
// 0.21 / 0.139 / 0.338 ms with 4 / 16 / 64 lanes.
int graph_auto_lanes(double mean_degree) {
    if (mean_degree < 3.0) return 1;
    if (mean_degree < 8.0) return 4;
    if (mean_degree < 256.0) return 16;
    return 64;
}

}  // namespace

}  // namespace flock

using namespace flock;

extern "C" {

int gr_opinion_step(int64_t n, int64_t n_edges, const int64_t *row_ptr, const int32_t *col,
                    const float *weight, float threshold, float strength, const float *op_in,
                    float *op_out, int lanes, void *stream) {
    if (n < 0 || n > INT32_MAX || n_edges < 0)
        return set_error(ENV_EINVAL, "need 0 <= n <= 2^31 - 1 and n_edges >= 0");
    if (!isfinite(threshold) || !isfinite(strength))
        return set_error(ENV_EINVAL, "threshold and strength must be finite");
    if (lanes != 0 && lanes != 1 && lanes != 4 && lanes != 16 && lanes != 64)
        return set_error(ENV_EINVAL, "lanes must be 0, 1, 4, 16 or 64");
    if (n == 0) return ENV_OK;
    if (!row_ptr || !op_in || !op_out || (n_edges > 0 && (!col || !weight)))
        return set_error(ENV_EINVAL, "NULL array");
    if (op_in == op_out) return set_error(ENV_EINVAL, "op_in and op_out must differ");
    const int g = lanes ? lanes : graph_auto_lanes((double)n_edges / (double)n);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const double st = (double)strength;
    auto run = [&](auto tag) {
        constexpr int G = decltype(tag)::value;
        launch_opinion<G>(n, n_edges, row_ptr, col, weight, threshold, st, op_in, op_out, s);
    };
    if (g == 1) run(std::integral_constant<int, 1>{});
    else if (g == 4) run(std::integral_constant<int, 4>{});
    else if (g == 16) run(std::integral_constant<int, 16>{});
    else run(std::integral_constant<int, 64>{});
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ENV_EHIP, "gr_opinion_step: %s", hipGetErrorString(e));
    return ENV_OK;
}

}  // extern "C"
