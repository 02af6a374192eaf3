// Batches of independent 1D/2D instances in one persistent launch.
//
// Each workgroup repeatedly takes the next task from a queue (a global
// counter; tasks are instances ordered by decreasing cost, so the largest
// start first) and runs every step of that instance before taking another.
// Instances whose field fits in LDS are stepped entirely in LDS (one global
// read and one write per launch).  Larger 2D ones advance in rounds of up to
// `depth` steps (1..8, autotuned; 4 by default) over 32 x 64 LDS regions or
// register-resident regions of 32 or 64 rows (autotuned; temporal blocking,
// one global read and write per round); larger 1D ones
// ping-pong between their two arena slots with a workgroup barrier between
// steps.  Every instance carries its own shape, boundary condition, kappa, h
// and Newton count, and every update uses the same arithmetic as the
// single-instance kernels, so each instance's result equals ace_step on that
// instance bit for bit.
//
// With register-resident regions the large 2D instances are queued for a
// kernel of their own (launched first, on the same stream), so that neither
// kernel carries the other's register pressure.  The launches (counter reset
// by a one-thread kernel, then the persistent kernels) are captured once per
// step count into a HIP graph and replayed.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ace.h"
#include "ace_device.h"
#include "ace_runtime.h"
#include "ace_tb2.h"
#include "ace_tile2d.h"

namespace ace {

struct BatchInst {
    int d, bc;
    int64_t M1, M2;   // 1D: 1 x M; 2D: M0 x M1 of the problem
    int64_t total;
    int64_t off;      // field offset in both arenas (doubles)
    StepCoef c;
    int resident;     // 1: stepped in LDS
};

namespace {

constexpr int kBT = 1024;                       // threads per workgroup
constexpr int kBNodes = (int)((RESIDENT_MAX + kBT - 1) / kBT);

template <int D, int BC>
__device__ void batch_resident(const BatchInst &I, double *__restrict__ fa, int64_t nsteps,
                               double *f)
{
    const int total = (int)I.total;
    const int tid = threadIdx.x;
    const int M1 = (int)I.M1, M2 = (int)I.M2;
    int nb_lo[kBNodes][2], nb_hi[kBNodes][2];
#pragma unroll
    for (int k = 0; k < kBNodes; ++k) {
        const int j = tid + k * kBT;
        const int jj = j < total ? j : 0;
        const int cc[2] = {jj / M2, jj % M2};
        const int n[2] = {M1, M2};
        const int st[2] = {M2, 1};
#pragma unroll
        for (int a = 2 - D; a < 2; ++a) {
            int lo, hi;
            if (cc[a] > 0) lo = j - st[a];
            else lo = (BC == BC_HN) ? j : (BC == BC_HD ? total : j + (n[a] - 1) * st[a]);
            if (cc[a] < n[a] - 1) hi = j + st[a];
            else hi = (BC == BC_HN) ? j : (BC == BC_HD ? total : j - (n[a] - 1) * st[a]);
            nb_lo[k][a] = lo;
            nb_hi[k][a] = hi;
        }
    }
    for (int j = tid; j < total; j += kBT) f[j] = fa[j];
    if (tid == 0) f[total] = 0.0;
    __syncthreads();
    for (int64_t step = 0; step < nsteps; ++step) {
        double nv[kBNodes];
#pragma unroll
        for (int k = 0; k < kBNodes; ++k) {
            const int j = tid + k * kBT;
            nv[k] = 0.0;
            if (j < total) {
                double nsum = 0.0;
#pragma unroll
                for (int a = 2 - D; a < 2; ++a) nsum += f[nb_lo[k][a]] + f[nb_hi[k][a]];
                nv[k] = update<D>(f[j], nsum, I.c);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kBNodes; ++k) {
            const int j = tid + k * kBT;
            if (j < total) f[j] = nv[k];
        }
        __syncthreads();
    }
    for (int j = tid; j < total; j += kBT) fa[j] = f[j];
    __syncthreads();
}

// Instance too large for LDS: one wavefront per 64-node segment of a row,
// neighbours through the cache, workgroup barrier (with its memory fence)
// between steps; the field ping-pongs between its two arena slots.
template <int D, int BC>
__device__ void batch_stream(const BatchInst &I, double *__restrict__ fa, double *__restrict__ fb,
                             int64_t nsteps)
{
    const int64_t M1 = I.M1, M2 = I.M2;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = kBT / 64;
    const int64_t nseg = (M2 + 63) / 64;
    for (int64_t step = 0; step < nsteps; ++step) {
        const double *__restrict__ in = (step & 1) ? fb : fa;
        double *__restrict__ out = (step & 1) ? fa : fb;
        for (int64_t r = wave; r < M1 * nseg; r += nw) {
            const int64_t i1 = r / nseg;
            const int64_t i2 = (r - i1 * nseg) * 64 + lane;
            if (i2 >= M2) continue;
            const int64_t idx = i1 * M2 + i2;
            const double p = in[idx];
            double nsum = 0.0;
            if (D == 2) {
                double ylo, yhi;
                if (i1 > 0) ylo = in[idx - M2];
                else ylo = outside<BC>(p, BC == BC_P ? in[idx + (M1 - 1) * M2] : 0.0);
                if (i1 < M1 - 1) yhi = in[idx + M2];
                else yhi = outside<BC>(p, BC == BC_P ? in[idx - (M1 - 1) * M2] : 0.0);
                nsum += ylo + yhi;
            }
            double xlo, xhi;
            if (i2 > 0) xlo = in[idx - 1];
            else xlo = outside<BC>(p, BC == BC_P ? in[idx + (M2 - 1)] : 0.0);
            if (i2 < M2 - 1) xhi = in[idx + 1];
            else xhi = outside<BC>(p, BC == BC_P ? in[idx - (M2 - 1)] : 0.0);
            nsum += xlo + xhi;
            out[idx] = update<D>(p, nsum, I.c);
        }
        __threadfence_block();
        __syncthreads();
    }
    if (nsteps & 1) {  // result back into the first arena
        for (int64_t j = threadIdx.x; j < M1 * M2; j += kBT) fa[j] = fb[j];
        __threadfence_block();
        __syncthreads();
    }
}

// 2D instance too large for LDS, advanced in rounds of up to tk steps (the
// batch's depth, 1..kMaxDepth): each round walks the instance's 32 x 64
// regions (ring of K nodes), advances each region K levels in LDS (the two
// padded planes live in the workgroup's LDS array) and writes its tile
// interior to the other arena slot; a workgroup barrier (with its memory
// fence) separates the rounds.  The arithmetic and neighbour order are those
// of the single-instance kernels.
constexpr int kMaxDepth = 8;

template <int BC>
__device__ void batch_tiles2d(const BatchInst &I, double *__restrict__ fa, double *__restrict__ fb,
                              int64_t nsteps, double *lds, int tk)
{
    using namespace tile2d;
    constexpr int TR = kBT / BX;  // thread rows
    constexpr int RT = BH / TR;   // region rows per thread
    static_assert(2 * BLP <= RESIDENT_MAX + 1, "two padded planes must fit the LDS array");
    Shape s;
    s.d = 2;
    s.bc = BC;
    s.M0 = 1;
    s.M1 = I.M1;
    s.M2 = I.M2;
    const int tx = threadIdx.x & (BX - 1), tr = threadIdx.x / BX;
    double *F = lds;
    for (int i = threadIdx.x; i < 2 * BLP; i += kBT) F[i] = 0.0;  // zero pads
    __syncthreads();
    int64_t done = 0;
    int par = 0;  // 0: the field is in fa
    while (done < nsteps) {
        const int K = (int)std::min<int64_t>(tk, nsteps - done);
        const double *__restrict__ in = par ? fb : fa;
        double *__restrict__ out = par ? fa : fb;
        const int64_t tiles_x = (s.M2 + BX - 2 * K - 1) / (BX - 2 * K);
        const int64_t tiles_y = (s.M1 + BH - 2 * K - 1) / (BH - 2 * K);
        const int64_t ntiles = tiles_x * tiles_y;
        // the next region's values are loaded into registers while the
        // current region advances, and staged after its last level
        double nxt[RT];
        auto fetch = [&](int64_t t) {
            const Geo gn = make_geo<BC>(s, K, tiles_x, t, tx);
#pragma unroll
            for (int j = 0; j < RT; ++j) {
                const int64_t o = goff<BC>(s, gn.y0r + tr + TR * j, gn.xg);
                nxt[j] = (o < 0) ? 0.0 : in[o];
            }
        };
        fetch(0);
        for (int64_t t = 0; t < ntiles; ++t) {
            const Geo g = make_geo<BC>(s, K, tiles_x, t, tx);
            const bool xin = g.xg >= 0 && g.xg < s.M2 && tx >= K && tx < BX - K;
#pragma unroll
            for (int j = 0; j < RT; ++j) F[(tr + TR * j + 1) * BLW + tx + 1] = nxt[j];
            __syncthreads();
            if (t + 1 < ntiles) fetch(t + 1);
            for (int k = 1; k <= K; ++k) {
                const double *src = F + ((k - 1) & 1) * BLP;
                double *dst = F + (k & 1) * BLP;
#pragma unroll
                for (int j = 0; j < RT; ++j) {
                    const int ry = tr + TR * j;
                    if (ry < k || ry >= BH - k) continue;  // wave-uniform
                    int ym, yp;
                    yoffs<BC>(s, g, ry, ym, yp);
                    const int o = (ry + 1) * BLW + tx + 1;
                    const double p = src[o];
                    const double nsum = (src[o + ym] + src[o + yp]) + (src[o + g.xm] + src[o + g.xp]);
                    const double v = update<2>(p, nsum, I.c);
                    dst[o] = v;
                    const int64_t yg = g.y0r + ry;
                    if (k == K && xin && ry >= K && ry < BH - K && yg >= 0 && yg < s.M1)
                        out[yg * s.M2 + g.xg] = v;
                }
                __syncthreads();
            }
        }
        __threadfence_block();
        __syncthreads();
        done += K;
        par ^= 1;
    }
    if (par) {  // result back into the first arena
        for (int64_t j = threadIdx.x; j < s.M1 * s.M2; j += kBT) fa[j] = fb[j];
        __threadfence_block();
        __syncthreads();
    }
}

// The same rounds over register-resident regions (ace_tb2.h): each thread
// holds RYT consecutive rows of a column of a (16 RYT) x 64 region, nodes
// outside the instance are its boundary images, and the workgroup's LDS array
// holds the regions' edge rows.  The next region's values are loaded while
// the current one advances.  RV: the instance's root variant (ace_device.h).
template <int BC, int RYT, int RV>
__device__ void batch_regions(const BatchInst &I, double *__restrict__ fa, double *__restrict__ fb,
                              int64_t nsteps, double *lds, int tk)
{
    constexpr int TRW = kBT / 64;  // 16 wavefronts
    using Rg = tb2::Region<BC, TRW, RYT>;
    Shape s;
    s.d = 2;
    s.bc = BC;
    s.M0 = 1;
    s.M1 = I.M1;
    s.M2 = I.M2;
    MonAcc m;
    mon_zero(m);
    const StepCoef c = coef_vgpr(I.c);
    int64_t done = 0;
    int par = 0;  // 0: the field is in fa
    while (done < nsteps) {
        const int K = (int)std::min<int64_t>(tk, nsteps - done);
        const double *__restrict__ in = par ? fb : fa;
        double *__restrict__ out = par ? fa : fb;
        const int oy = Rg::RH - 2 * K, ox = 64 - 2 * K;
        const int tiles_x = ((int)s.M2 + ox - 1) / ox, tiles_y = ((int)s.M1 + oy - 1) / oy;
        double v[RYT], vn[RYT];
        Rg(s, K, 0, 0).load(s, in, v);
#pragma unroll
        for (int r = 0; r < RYT; ++r) vn[r] = 0.0;
        // regions row by row; the next one's values load while this one advances
        for (int ty = 0, tx = 0; ty < tiles_y;) {
            const Rg g(s, K, ty, tx);
            int nty = ty, ntx = tx + 1;
            if (ntx == tiles_x) {
                ntx = 0;
                ++nty;
            }
            if (nty < tiles_y) Rg(s, K, nty, ntx).load(s, in, vn);
            g.template advance<false, false, RV>(s, c, v, out, 0, lds, m);
            __syncthreads();  // every wavefront is past the edge rows before the next region writes them
#pragma unroll
            for (int r = 0; r < RYT; ++r) v[r] = vn[r];
            ty = nty;
            tx = ntx;
        }
        __threadfence_block();
        __syncthreads();
        done += K;
        par ^= 1;
    }
    if (par) {  // result back into the first arena
        for (int64_t j = threadIdx.x; j < s.M1 * s.M2; j += kBT) fa[j] = fb[j];
        __threadfence_block();
        __syncthreads();
    }
}

__global__ void k_batch_reset(int *counter)
{
    if (threadIdx.x < 2 && blockIdx.x == 0) counter[threadIdx.x] = 0;
}

// The tasks order[first .. last) taken from the queue counter.  REGION = 0:
// every kind of instance (large 2D ones over LDS-plane regions); 32 or 64:
// large 2D instances only, over register-resident regions of that height.
template <int REGION>
__global__ __launch_bounds__(kBT) void k_batch(const BatchInst *__restrict__ inst,
                                               const int *__restrict__ order, int first, int last,
                                               int *__restrict__ counter, double *__restrict__ arena_a,
                                               double *__restrict__ arena_b, int64_t nsteps, int tk)
{
    __shared__ double f[REGION ? 2 * 2 * (kBT / 64) * 64 : RESIDENT_MAX + 1];
    __shared__ int task;
    for (;;) {
        if (threadIdx.x == 0) task = first + atomicAdd(counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(task);
        __syncthreads();  // all threads read the task before the next fetch
        if (t >= last) break;
        const BatchInst I = inst[order[t]];
        double *fa = arena_a + I.off;
        double *fb = arena_b + I.off;
        if (REGION != 0) {
            constexpr int RYT = REGION == 64 ? 4 : 2;
            auto by_rv = [&](auto BCc) {
                constexpr int B = decltype(BCc)::value;
                // every root variant with an instantiation compiled in (the
                // explicit scheme and more than 3 Newton steps: the run-time root)
                switch (root_variant(I.c)) {
                case 1: batch_regions<B, RYT, 1>(I, fa, fb, nsteps, f, tk); break;
                case 2: batch_regions<B, RYT, 2>(I, fa, fb, nsteps, f, tk); break;
                case 3: batch_regions<B, RYT, 3>(I, fa, fb, nsteps, f, tk); break;
                case 5: batch_regions<B, RYT, 5>(I, fa, fb, nsteps, f, tk); break;
                case 6: batch_regions<B, RYT, 6>(I, fa, fb, nsteps, f, tk); break;
                default: batch_regions<B, RYT, 0>(I, fa, fb, nsteps, f, tk); break;
                }
            };
            if (I.bc == BC_HN) by_rv(std::integral_constant<int, BC_HN>());
            else if (I.bc == BC_HD) by_rv(std::integral_constant<int, BC_HD>());
            else by_rv(std::integral_constant<int, BC_P>());
        } else if (I.resident) {
            if (I.d == 1) {
                if (I.bc == BC_HN) batch_resident<1, BC_HN>(I, fa, nsteps, f);
                else if (I.bc == BC_HD) batch_resident<1, BC_HD>(I, fa, nsteps, f);
                else batch_resident<1, BC_P>(I, fa, nsteps, f);
            } else {
                if (I.bc == BC_HN) batch_resident<2, BC_HN>(I, fa, nsteps, f);
                else if (I.bc == BC_HD) batch_resident<2, BC_HD>(I, fa, nsteps, f);
                else batch_resident<2, BC_P>(I, fa, nsteps, f);
            }
        } else if (I.d == 1) {
            if (I.bc == BC_HN) batch_stream<1, BC_HN>(I, fa, fb, nsteps);
            else if (I.bc == BC_HD) batch_stream<1, BC_HD>(I, fa, fb, nsteps);
            else batch_stream<1, BC_P>(I, fa, fb, nsteps);
        } else {
            if (I.bc == BC_HN) batch_tiles2d<BC_HN>(I, fa, fb, nsteps, f, tk);
            else if (I.bc == BC_HD) batch_tiles2d<BC_HD>(I, fa, fb, nsteps, f, tk);
            else batch_tiles2d<BC_P>(I, fa, fb, nsteps, f, tk);
        }
    }
}

// Monitor triple (bulk, grad, max) of each instance: one workgroup each.
__global__ __launch_bounds__(256) void k_batch_monitor(const BatchInst *__restrict__ inst,
                                                       const double *__restrict__ arena_a,
                                                       double *__restrict__ trip)
{
    __shared__ double lds[3 * 4];
    const BatchInst I = inst[blockIdx.x];
    const double *f = arena_a + I.off;
    MonAcc m;
    mon_zero(m);
    for (int64_t j = threadIdx.x; j < I.total; j += blockDim.x) {
        const int64_t i1 = j / I.M2, i2 = j - i1 * I.M2;
        const double p = f[j];
        double g = 0.0;
        const int64_t cc[2] = {i1, i2};
        const int64_t n[2] = {I.M1, I.M2};
        const int64_t st[2] = {I.M2, 1};
        for (int a = 2 - I.d; a < 2; ++a) {
            double hi;
            if (cc[a] < n[a] - 1) hi = f[j + st[a]];
            else hi = (I.bc == BC_HN) ? p : (I.bc == BC_HD ? 0.0 : f[j - (n[a] - 1) * st[a]]);
            const double dh = hi - p;
            g = fma(dh, dh, g);
            if (I.bc == BC_HD && cc[a] == 0) g = fma(p, p, g);
        }
        m.bulk += bulk_term(p);
        m.grad += g;
        m.mx = nan_max(m.mx, fabs(p));
    }
    block_reduce_store(m, lds, trip + 3 * blockIdx.x);
}

}  // namespace
}  // namespace ace

using namespace ace;

struct ace_batch {
    int count = 0;
    std::vector<Problem> prob;
    std::vector<BatchInst> host_inst;
    std::vector<int> order;
    int64_t arena_total = 0;
    int64_t resident_limit = RESIDENT_MAX;  // tuned: largest field stepped in LDS
    int depth = 4;  // tuned: steps per round of the 2D instances stepped over LDS regions
    int region = 0;  // tuned: 0 LDS-plane 32 x 64 regions; 32 or 64: register-resident regions of that height
    int device = 0;
    hipStream_t stream = nullptr;   // caller's stream (graph launches go here)
    hipStream_t capture = nullptr;  // private stream used only for graph capture
    BatchInst *inst = nullptr;
    int *order_dev = nullptr;
    int *counter = nullptr;  // [0] queue of the first kernel, [1] of the second
    int n_large = 0;         // order[0 .. n_large): 2D instances too large for LDS (32-bit indexable)
    double *arena_a = nullptr, *arena_b = nullptr;
    double *trip = nullptr;
    int grid = 0;     // workgroups of the queue kernel
    int grid_rg = 0;  // workgroups of the register-region kernels
    int use_graphs = 1;  // 0: the launch pair is issued directly on every step call
    std::map<int64_t, hipGraphExec_t> graphs;
    std::map<int64_t, hipGraph_t> graph_defs;
};

namespace {

#define BT_TRY(expr)            \
    do {                        \
        const int _rc = (expr); \
        if (_rc < 0) return _rc; \
    } while (0)
#define BT_HIP(expr) BT_TRY(hip_status(expr))

void drop_graphs(ace_batch *b)
{
    // a replay may still run on the handle's stream
    if (!b->graphs.empty()) (void)hipStreamSynchronize(b->stream);
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : b->graph_defs) (void)hipGraphDestroy(kv.second);
    b->graphs.clear();
    b->graph_defs.clear();
}

// Cost model for the queue order: node updates, with streaming instances
// weighted by their extra memory traffic.
int64_t task_cost(const BatchInst &I) { return I.total * (I.resident ? 1 : 3); }

int upload_tasks(ace_batch *b)
{
    // the tables below are read by any launch still running on the stream
    BT_HIP(hipStreamSynchronize(b->stream));
    for (auto &I : b->host_inst) I.resident = (I.total <= b->resident_limit) ? 1 : 0;
    // the large 2D instances first (the register-region kernel's queue; the
    // regions index a field with 32 bits), then the rest, each by cost
    auto large = [&](int x) {
        const BatchInst &I = b->host_inst[x];
        return I.d == 2 && !I.resident && I.total <= INT32_MAX;
    };
    b->order.resize(b->count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        if (large(x) != large(y)) return large(x);
        return task_cost(b->host_inst[x]) > task_cost(b->host_inst[y]);
    });
    b->n_large = (int)std::count_if(b->order.begin(), b->order.end(), large);
    BT_HIP(hipMemcpy(b->inst, b->host_inst.data(), sizeof(BatchInst) * b->count,
                     hipMemcpyHostToDevice));
    BT_HIP(hipMemcpy(b->order_dev, b->order.data(), sizeof(int) * b->count, hipMemcpyHostToDevice));
    drop_graphs(b);
    return ACE_OK;
}

// The batch kernels for the chosen region, on stream st (the counters must
// be zero): the register-region kernel over the large 2D instances, then the
// queue kernel over the rest; or the queue kernel over every instance.
void launch_batch(const ace_batch *b, hipStream_t st, int64_t nsteps)
{
    auto go = [&](auto kern, int grid, int first, int last, int q) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kBT), 0, st, b->inst, b->order_dev, first, last, b->counter + q,
                           b->arena_a, b->arena_b, nsteps, b->depth);
    };
    int first = 0;
    if (b->region != 0 && b->n_large > 0) {
        if (b->region == 64) go(k_batch<64>, b->grid_rg, 0, b->n_large, 0);
        else go(k_batch<32>, b->grid_rg, 0, b->n_large, 0);
        first = b->n_large;
    }
    if (first < b->count) go(k_batch<0>, b->grid, first, b->count, 1);
}

int get_graph(ace_batch *b, int64_t nsteps, hipGraphExec_t *out)
{
    auto it = b->graphs.find(nsteps);
    if (it != b->graphs.end()) {
        *out = it->second;
        return ACE_OK;
    }
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    BT_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->capture, b->counter);
    launch_batch(b, b->capture, nsteps);
    hipError_t le = hipGetLastError();
    hipError_t ce = hipStreamEndCapture(b->capture, &g);
    BT_HIP(le);
    BT_HIP(ce);
    hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_status(ie);
    }
    b->graphs[nsteps] = e;
    b->graph_defs[nsteps] = g;
    *out = e;
    return ACE_OK;
}

}  // namespace

extern "C" {

int ace_batch_create(int count, const ace_instance_desc *desc, ace_batch **out, int *status)
{
    if (!out || !desc || count < 1) return ACE_E_ARG;
    *out = nullptr;
    ace_batch *b = new (std::nothrow) ace_batch();
    if (!b) return ACE_E_NOMEM;
    b->count = count;
    b->prob.resize(count);
    b->host_inst.resize(count);
    int worst = ACE_OK, warn = ACE_OK;
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
        const ace_instance_desc &D = desc[i];
        int rc = (D.d == 1 || D.d == 2) ? derive(D.d, D.N, D.L, D.R, D.eps, D.dt, D.bc, b->prob[i])
                                        : ACE_E_ARG;
        if (status) status[i] = rc;
        if (rc < 0 && worst == ACE_OK) worst = rc;
        if (rc > 0) warn = rc;
        if (rc < 0) continue;
        const Problem &p = b->prob[i];
        BatchInst &I = b->host_inst[i];
        I.d = p.d;
        I.bc = p.bc;
        I.M1 = (p.d == 1) ? 1 : p.M[0];
        I.M2 = (p.d == 1) ? p.M[0] : p.M[1];
        I.total = p.total;
        I.off = off;
        I.c = coef_of(p);
        I.resident = 0;
        off += (p.total + 31) / 32 * 32;  // 256-byte aligned fields
    }
    if (worst < 0) {
        delete b;
        return worst;
    }
    b->arena_total = off;
    (void)hipGetDevice(&b->device);
    int rc = ACE_OK;
    auto fail = [&](int r) {
        ace_batch_destroy(b);
        return r;
    };
    if ((rc = hip_status(hipMalloc((void **)&b->arena_a, sizeof(double) * off))) < 0) return fail(rc);
    if ((rc = hip_status(hipMalloc((void **)&b->arena_b, sizeof(double) * off))) < 0) return fail(rc);
    if ((rc = hip_status(hipMemset(b->arena_a, 0, sizeof(double) * off))) < 0) return fail(rc);
    if ((rc = hip_status(hipMalloc((void **)&b->inst, sizeof(BatchInst) * count))) < 0) return fail(rc);
    if ((rc = hip_status(hipMalloc((void **)&b->order_dev, sizeof(int) * count))) < 0) return fail(rc);
    if ((rc = hip_status(hipMalloc((void **)&b->counter, sizeof(int) * 64))) < 0) return fail(rc);
    if ((rc = hip_status(hipMalloc((void **)&b->trip, sizeof(double) * 3 * count))) < 0) return fail(rc);
    if ((rc = hip_status(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking))) < 0) return fail(rc);
    int cus = 0, per_cu = 0;
    if ((rc = hip_status(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                               b->device))) < 0)
        return fail(rc);
    if ((rc = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<0>, kBT, 0))) < 0)
        return fail(rc);
    b->grid = std::max(1, cus * std::max(1, per_cu));
    int per_cu_rg = 0, per_cu_rg32 = 0;
    if ((rc = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_rg, k_batch<64>, kBT, 0))) < 0 ||
        (rc = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_rg32, k_batch<32>, kBT, 0))) < 0)
        return fail(rc);
    b->grid_rg = std::max(1, cus * std::max(1, std::min(per_cu_rg, per_cu_rg32)));
    if ((rc = upload_tasks(b)) < 0) return fail(rc);
    *out = b;
    return warn;
}

int ace_batch_destroy(ace_batch *b)
{
    if (!b) return ACE_E_ARG;
    drop_graphs(b);
    void *ptrs[] = {b->arena_a, b->arena_b, b->inst, b->order_dev, b->counter, b->trip};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
    return ACE_OK;
}

int ace_batch_shape(const ace_batch *b, int i, int64_t M[3], int64_t *total, int64_t *offset)
{
    if (!b || i < 0 || i >= b->count) return ACE_E_ARG;
    const Problem &p = b->prob[i];
    if (M)
        for (int j = 0; j < 3; ++j) M[j] = p.M[j];
    if (total) *total = p.total;
    if (offset) *offset = b->host_inst[i].off;
    return ACE_OK;
}

int ace_batch_set_stream(ace_batch *b, void *st)
{
    if (!b) return ACE_E_ARG;
    // a replay on the old stream may still use a captured graph
    if ((hipStream_t)st != b->stream) drop_graphs(b);
    b->stream = (hipStream_t)st;
    return ACE_OK;
}

int ace_batch_set_phi0(ace_batch *b, int i, const double *phi0, int where)
{
    if (!b || !phi0 || i < 0 || i >= b->count || (where != ACE_HOST && where != ACE_DEVICE))
        return ACE_E_ARG;
    const BatchInst &I = b->host_inst[i];
    int warn = ACE_OK;
    if (where == ACE_HOST) {
        for (int64_t j = 0; j < I.total; ++j) {
            if (!isfinite(phi0[j])) return ACE_E_NONFINITE;
            if (fabs(phi0[j]) > 1.0) warn = ACE_W_PHI0_GT1;
        }
    }
    BT_HIP(hipMemcpyAsync(b->arena_a + I.off, phi0, sizeof(double) * I.total,
                          where == ACE_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                          b->stream));
    if (where == ACE_HOST) BT_HIP(hipStreamSynchronize(b->stream));
    return warn;
}

int ace_batch_set_all(ace_batch *b, const double *all, int where)
{
    if (!b || !all || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    int64_t src = 0;
    int warn = ACE_OK;
    for (int i = 0; i < b->count; ++i) {
        const int rc = ace_batch_set_phi0(b, i, all + src, where);
        if (rc < 0) return rc;
        if (rc > 0) warn = rc;
        src += b->host_inst[i].total;
    }
    return warn;
}

int ace_batch_step(ace_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0) return ACE_E_ARG;
    if (nsteps == 0) return ACE_OK;
    if (!b->use_graphs) {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->stream, b->counter);
        launch_batch(b, b->stream, nsteps);
        BT_HIP(hipGetLastError());
        return ACE_OK;
    }
    hipGraphExec_t e = nullptr;
    BT_TRY(get_graph(b, nsteps, &e));
    BT_HIP(hipGraphLaunch(e, b->stream));
    return ACE_OK;
}

int ace_batch_set_region(ace_batch *b, int rows)
{
    if (!b || (rows != 0 && rows != 32 && rows != 64)) return ACE_E_ARG;
    if (rows != b->region) {
        b->region = rows;
        drop_graphs(b);  // the captured launches carry the old region
    }
    return ACE_OK;
}

int ace_batch_set_graphs(ace_batch *b, int enable)
{
    if (!b || (enable != 0 && enable != 1)) return ACE_E_ARG;
    b->use_graphs = enable;
    return ACE_OK;
}

int ace_batch_monitor(ace_batch *b, double *E, double *maxn)
{
    if (!b || !E || !maxn) return ACE_E_ARG;
    hipLaunchKernelGGL(k_batch_monitor, dim3(b->count), dim3(256), 0, b->stream, b->inst,
                       b->arena_a, b->trip);
    BT_HIP(hipGetLastError());
    std::vector<double> t(3 * (size_t)b->count);
    BT_HIP(hipMemcpyAsync(t.data(), b->trip, sizeof(double) * t.size(), hipMemcpyDeviceToHost,
                          b->stream));
    BT_HIP(hipStreamSynchronize(b->stream));
    int rc = ACE_OK;
    for (int i = 0; i < b->count; ++i) {
        E[i] = energy_from(b->prob[i], &t[3 * i]);
        maxn[i] = t[3 * i + 2];
        if (!isfinite(E[i]) || !isfinite(maxn[i])) rc = ACE_E_NONFINITE;
    }
    return rc;
}

int ace_batch_get_phi(ace_batch *b, int i, double *out, int where)
{
    if (!b || !out || i < 0 || i >= b->count || (where != ACE_HOST && where != ACE_DEVICE))
        return ACE_E_ARG;
    const BatchInst &I = b->host_inst[i];
    BT_HIP(hipMemcpyAsync(out, b->arena_a + I.off, sizeof(double) * I.total,
                          where == ACE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                          b->stream));
    if (where == ACE_HOST) BT_HIP(hipStreamSynchronize(b->stream));
    return ACE_OK;
}

int ace_batch_get_all(ace_batch *b, double *out, int where)
{
    if (!b || !out) return ACE_E_ARG;
    int64_t dst = 0;
    for (int i = 0; i < b->count; ++i) {
        const int rc = ace_batch_get_phi(b, i, out + dst, where);
        if (rc < 0) return rc;
        dst += b->host_inst[i].total;
    }
    return ACE_OK;
}

int ace_batch_set_resident_limit(ace_batch *b, int64_t limit)
{
    if (!b || limit < 0) return ACE_E_ARG;
    b->resident_limit = std::min<int64_t>(limit, RESIDENT_MAX);
    return upload_tasks(b);
}

int ace_batch_set_depth(ace_batch *b, int depth)
{
    if (!b || depth < 1 || depth > kMaxDepth) return ACE_E_ARG;
    if (depth != b->depth) {
        b->depth = depth;
        drop_graphs(b);  // the captured launches carry the old depth
    }
    return ACE_OK;
}

int ace_batch_autotune(ace_batch *b, int64_t trial_steps, char *json, size_t cap)
{
    if (!b || trial_steps < 1) return ACE_E_ARG;
    // keep the current fields: time each candidate on a copy, then restore
    double *save = nullptr;
    BT_HIP(hipMalloc((void **)&save, sizeof(double) * b->arena_total));
    auto restore = [&]() {
        return hip_status(hipMemcpyAsync(b->arena_a, save, sizeof(double) * b->arena_total,
                                         hipMemcpyDeviceToDevice, b->stream));
    };
    int rc = hip_status(hipMemcpyAsync(save, b->arena_a, sizeof(double) * b->arena_total,
                                       hipMemcpyDeviceToDevice, b->stream));
    // First the region shape and depth of the region rounds at the current
    // resident limit, then the resident limit at the chosen pair.
    const int depths[] = {2, 3, 4, 5, 6};
    const int regions[] = {0, 32, 64};
    const int64_t limits[] = {0, 1024, 2048, 4096, RESIDENT_MAX};
    double best_ms = 1e300;
    int64_t best_lim = b->resident_limit;
    int best_depth = b->depth;
    int best_region = b->region;
    std::string rec = "{\"kind\": \"batch\", \"trial_steps\": " + std::to_string(trial_steps) +
                      ", \"workgroups\": " + std::to_string(b->grid) +
                      ", \"workgroups_regions\": " + std::to_string(b->grid_rg) + ", \"candidates\": [";
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc >= 0) rc = hip_status(hipEventCreate(&e0));
    if (rc >= 0) rc = hip_status(hipEventCreate(&e1));
    bool first = true;
    // times one batch step of trial_steps for (lim, depth, region); returns ms or a negative error
    auto trial = [&](int64_t lim, int depth, int region, double *ms_out) -> int {
        int r;
        if ((r = ace_batch_set_resident_limit(b, lim)) < 0) return r;
        if ((r = ace_batch_set_depth(b, depth)) < 0) return r;
        if ((r = ace_batch_set_region(b, region)) < 0) return r;
        if ((r = restore()) < 0) return r;
        if ((r = ace_batch_step(b, trial_steps)) < 0) return r;  // builds the graph, warms up
        if ((r = restore()) < 0) return r;
        if ((r = hip_status(hipEventRecord(e0, b->stream))) < 0) return r;
        if ((r = ace_batch_step(b, trial_steps)) < 0) return r;
        if ((r = hip_status(hipEventRecord(e1, b->stream))) < 0) return r;
        if ((r = hip_status(hipEventSynchronize(e1))) < 0) return r;
        float ms = 0.f;
        if ((r = hip_status(hipEventElapsedTime(&ms, e0, e1))) < 0) return r;
        *ms_out = ms;
        char buf[160];
        snprintf(buf, sizeof buf, "%s{\"resident_limit\": %lld, \"depth\": %d, \"region\": %d, \"ms\": %.4f}",
                 first ? "" : ", ", (long long)lim, depth, region, ms);
        rec += buf;
        first = false;
        return ACE_OK;
    };
    const int64_t lim0 = b->resident_limit;
    for (int region : regions)
        for (int depth : depths) {
            if (rc < 0) break;
            double ms = 0.0;
            if ((rc = trial(lim0, depth, region, &ms)) < 0) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_depth = depth;
                best_region = region;
                best_lim = lim0;
            }
        }
    for (int64_t lim : limits) {
        if (rc < 0) break;
        if (lim == lim0) continue;  // timed above at the chosen depth
        double ms = 0.0;
        if ((rc = trial(lim, best_depth, best_region, &ms)) < 0) break;
        if (ms < best_ms) {
            best_ms = ms;
            best_lim = lim;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc >= 0) rc = ace_batch_set_resident_limit(b, best_lim);
    if (rc >= 0) rc = ace_batch_set_depth(b, best_depth);
    if (rc >= 0) rc = ace_batch_set_region(b, best_region);
    if (rc >= 0) rc = restore();
    if (rc >= 0) rc = hip_status(hipStreamSynchronize(b->stream));
    (void)hipFree(save);
    if (rc < 0) return rc;
    rec += "], \"choice\": {\"resident_limit\": " + std::to_string(best_lim) +
           ", \"depth\": " + std::to_string(best_depth) + ", \"region\": " + std::to_string(best_region) + "}}";
    if (log_enabled())
        fprintf(stderr,
                "[ace] batch autotune (%d instances): LDS limit %lld nodes, region depth %d, region rows %d, "
                "%.4f ms\n",
                b->count, (long long)best_lim, best_depth, best_region, best_ms);
    if (json && cap > 0) snprintf(json, cap, "%s", rec.c_str());
    return ACE_OK;
}

}  // extern "C"
