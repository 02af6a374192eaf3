// Host runtime behind the C ABI declared in include/ace.h: argument checks,
// derived parameters (Sec. 2; Theorem 2 of Sec. 3.2), device buffers, kernel
// dispatch, monitored runs, and the checkpointed reverse sweep.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ace.h"
#include "ace_internal.h"
#include "ace_runtime.h"

using namespace ace;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

namespace ace {

bool log_enabled()
{
    static const bool on = getenv("ACE_LOG") != nullptr;
    return on;
}

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return ACE_OK;
    if (e == hipErrorOutOfMemory) return ACE_E_NOMEM;
    if (log_enabled()) fprintf(stderr, "[ace] HIP error: %s\n", hipGetErrorString(e));
    return ACE_E_HIP;
}

int64_t nodes_per_axis(int64_t N, int bc)
{
    if (bc == ACE_BC_HN) return N + 2;
    if (bc == ACE_BC_HD) return N - 1;
    return N;
}

// Newton steps of the device root (ace_device.h, cubic_root) needed for
// |xi| <= 1: the same start (theta_0 = a + h a (1 - a^2) for h <= 1/2, else
// theta_0 = a) and the same Newton
// step are run in long double on a grid of a in (0, 1]; nit is the first step
// count whose largest relative error against the converged root is below
// 2^-60 (well under half an ulp, leaving room for the reciprocal estimate and
// the rounding of the double iteration).
int newton_iters_for(double h, int start2)
{
    const long double H = h;
    const int G = 2048;
    int need = 1;
    for (int j = 1; j <= G + 8; ++j) {
        long double a = (j <= G) ? (long double)j / G : 1.0L - ldexpl(1.0L, -(j - G) * 6);
        long double ref = a;
        for (int k = 0; k < 200; ++k) {
            const long double p = ref + H * (ref * ref * ref - ref) - a;
            const long double dp = 1.0L + H * (3.0L * ref * ref - 1.0L);
            const long double nx = ref - p / dp;
            if (nx == ref) break;
            ref = nx;
        }
        long double x = a;
        if (H <= 0.5L) {
            const long double f = a * a * a - a;
            x = start2 ? a - H * f * (1.0L - H * (3.0L * a * a - 1.0L)) : a + H * a * (1.0L - a * a);
        }
        int k = 0;
        while (fabsl(x - ref) > ldexpl(ref, -60) && k < 60) {
            const long double p = x + H * (x * x * x - x) - a;
            const long double dp = 1.0L + H * (3.0L * x * x - 1.0L);
            x -= p / dp;
            ++k;
        }
        if (k > need) need = k;
    }
    return need;
}

// Theorem 2's step condition dt <= 1 - 2 d kappa, 0 < kappa < 1/(2d) (with
// 1e-12 relative slack for the equality case); for the explicit comparison
// scheme Remark 2's dt <= (1 - 2 d kappa)/2.
void set_conditions(Problem &p)
{
    double bound = 1.0 - 2.0 * p.d * p.kappa;
    if (p.scheme == ACE_SCHEME_FEX) bound *= 0.5;
    p.cond_ok = (p.dt <= bound * (1.0 + 1e-12)) && p.kappa > 0.0 && p.kappa < 1.0 / (2.0 * p.d);
}

// Validates the ace_create arguments and fills the derived parameters.
int derive(int d, const int64_t *N, const double *L, const double *R, double eps, double dt,
           int bc, Problem &p)
{
    if (!N || !L || !R) return ACE_E_ARG;
    if (d < 1 || d > 3) return ACE_E_ARG;
    if (bc != ACE_BC_HN && bc != ACE_BC_HD && bc != ACE_BC_P) return ACE_E_ARG;
    if (!(eps > 0.0) || !isfinite(eps)) return ACE_E_ARG;
    if (!isfinite(dt)) return ACE_E_ARG;
    const int64_t minN = (bc == ACE_BC_HN) ? 1 : (bc == ACE_BC_HD ? 2 : 3);
    memset(&p, 0, sizeof(p));
    p.d = d;
    p.bc = bc;
    for (int j = 0; j < 3; ++j) {
        p.N[j] = 1;
        p.M[j] = 1;
        p.L[j] = 0.0;
        p.R[j] = 1.0;
    }
    double dx0 = 0.0;
    for (int j = 0; j < d; ++j) {
        if (!isfinite(L[j]) || !isfinite(R[j]) || !(L[j] < R[j])) return ACE_E_ARG;
        if (N[j] < minN) return ACE_E_SIZE;
        if (N[j] > (int64_t)1 << 31) return ACE_E_SIZE;
        const double dx = (R[j] - L[j]) / (double)N[j];
        if (j == 0) dx0 = dx;
        else if (fabs(dx - dx0) > 1e-12 * dx0) return ACE_E_ANISO;
        p.N[j] = N[j];
        p.L[j] = L[j];
        p.R[j] = R[j];
    }
    if (!(dt > 0.0) || !(dt < 2.0)) return ACE_E_DT;
    p.dx = dx0;
    p.dt = dt;
    p.eps = eps;
    // kappa = eps^2 dt / dx^2 (Sec. 2: eps^2 = (omega_1/s) dx^2 / dt)
    p.kappa = eps * eps * dt / (dx0 * dx0);
    p.h = 0.5 * dt;
    // stored nodes: fastest axis last; a d-dimensional field occupies the
    // last d of the three internal axes
    int64_t total = 1;
    for (int j = 0; j < d; ++j) {
        const int64_t m = nodes_per_axis(N[j], bc);
        p.M[j] = m;
        total *= m;
    }
    p.total = total;
    // the second-order start costs two FMAs more and is used where it saves
    // Newton steps (e.g. one step instead of two for 1e-3 <= dt <= 5e-3)
    p.nit = newton_iters_for(p.h, 0);
    p.start2 = 0;
    const int nit2 = newton_iters_for(p.h, 1);
    if (nit2 < p.nit) {
        p.nit = nit2;
        p.start2 = 1;
    }
    p.scheme = ACE_SCHEME_RLB_MIE;
    set_conditions(p);
    return p.cond_ok ? ACE_OK : ACE_W_CONDITIONS;
}

Shape shape_of(const Problem &p)
{
    Shape s;
    s.d = p.d;
    s.bc = p.bc;
    if (p.d == 1) {
        s.M0 = 1;
        s.M1 = 1;
        s.M2 = p.M[0];
    } else if (p.d == 2) {
        s.M0 = 1;
        s.M1 = p.M[0];
        s.M2 = p.M[1];
    } else {
        s.M0 = p.M[0];
        s.M1 = p.M[1];
        s.M2 = p.M[2];
    }
    return s;
}

StepCoef coef_of(const Problem &p)
{
    StepCoef c;
    c.kappa = p.kappa;
    c.h = p.h;
    c.omh = 1.0 - p.h;
    c.oph = 1.0 + p.h;
    c.h3 = 3.0 * p.h;
    c.hs = p.h > 0.5 ? 0.0 : p.h;
    c.nit = p.nit;
    c.start2 = p.start2;
    c.fex = (p.scheme == ACE_SCHEME_FEX) ? 1 : 0;
    c.dt = p.dt;
    return c;
}

void energy_coefs(const Problem &p, double *dxd, double *cg)
{
    *dxd = pow(p.dx, p.d);
    *cg = p.kappa / (2.0 * p.dt);
}

double energy_from(const Problem &p, const double *trip)
{
    // E = dx^d [ sum (phi^2-1)^2/4 + kappa/(2 dt) sum_edges (dphi)^2 ]
    double dxd, cg;
    energy_coefs(p, &dxd, &cg);
    return dxd * (trip[0] + cg * trip[1]);
}

int grow(double **ptr, int64_t *cap, int64_t need)
{
    if (*cap >= need && *ptr) return ACE_OK;
    if (*ptr) (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc((void **)ptr, (size_t)need * sizeof(double));
    if (e != hipSuccess) {
        *ptr = nullptr;
        return hip_status(e);
    }
    *cap = need;
    return ACE_OK;
}

}  // namespace ace

// ---------------------------------------------------------------------------
// allocation-free monitor: device scratch held in a static array
// ---------------------------------------------------------------------------

namespace {

// Doubles of the static scratch: the reduced triple (kTripSlot doubles, so
// the partials that follow stay 256-byte aligned) and up to kNoAllocParts
// partial triples, 1.5 MiB per device for the life of the process.
constexpr int64_t kTripSlot = 32;
constexpr int64_t kNoAllocParts = 65536;
constexpr int64_t kNoAllocDoubles = kTripSlot + 3 * kNoAllocParts;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocDoubles];

// Device address of `scratch` on each device (host code must not pass the
// array's name: on the host it is only a stand-in for the symbol).
double *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Looks up the scratch address of the current device once; called by
// ace_create with the handle's device current.
void scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();  // leave no error behind for later launches
        if (log_enabled())
            fprintf(stderr, "[ace] scratch lookup on device %d failed: %s\n", dev, hipGetErrorString(e));
        return;
    }
    g_scratch[dev] = (double *)ptr;
}

double *scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

}  // namespace

#define ACE_TRY(expr)                  \
    do {                               \
        const int _rc = (expr);        \
        if (_rc < 0) return _rc;       \
    } while (0)
#define ACE_HIP(expr) ACE_TRY(hip_status(expr))

// ---------------------------------------------------------------------------
// solver handle
// ---------------------------------------------------------------------------

struct ace_solver {
    Problem p;
    Shape shape;
    StepCoef coef;
    int device = 0;
    hipStream_t stream = nullptr;
    double *own[2] = {nullptr, nullptr};
    double *buf[2] = {nullptr, nullptr};
    int cur = 0;
    double *partials = nullptr;
    int64_t partials_cap = 0;
    double *mon = nullptr;  // device monitor triples
    int64_t mon_cap = 0;
    double *pinned = nullptr;  // host pinned scratch (3 doubles)
    int64_t steps = 0;
    int warn_mask = 0;  // warnings of the last monitored run (ACE_WARN_BIT)
    int kernel = ACE_KERNEL_AUTO;
    int depth = 0;
    int zchunk = 32;  // planes per workgroup of the 3D temporal-blocking kernel (0: persistent)
    int depth2 = 5;   // steps per launch of the 2D temporal-blocking kernel (fastest on 1024^2)
    int tb3 = -1;     // variant of the configurable 3D blocked kernel (-1: the two-step kernel)
    int tb2 = -1;     // variant of the register-resident 2D blocked kernel (-1: the LDS-plane kernel)
    int tuned_kernel = 0;  // autotuned choice for ACE_KERNEL_AUTO (0: none)
    // reverse mode
    double *ckpt = nullptr;
    int64_t ckpt_cap = 0;
    int64_t ck_every = 0, ck_steps = 0, ck_count = 0;
    int64_t ck_field_version = -1;
    int64_t ck_generation = 0;  // incremented by every ace_forward_ckpt
    double *seg = nullptr;  // two segment buffers, (every + 1) states each
    int64_t seg_cap = 0;
    hipStream_t aux = nullptr;  // recompute stream of the pipelined reverse sweep
    hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
    double *lam = nullptr;
    int64_t lam_cap = 0;
    double *gpart = nullptr;
    int64_t gpart_cap = 0;
    double *gsum = nullptr;
    int64_t field_version = 0;
    // graph replay of runs of launches (0 disables)
    int64_t graph_launches = 32;
    hipStream_t capture = nullptr;
    struct GraphEntry {
        int kernel, zchunk, depth2, tb3, tb2, cur;
        const double *b0, *b1;
        hipGraph_t g;
        hipGraphExec_t e;
    };
    std::vector<GraphEntry> graphs;
};

namespace {

bool tblock_applies(const ace_solver *s)
{
    return (s->p.d == 3 && tblock_supported(s->shape)) || (s->p.d == 2 && tblock2d_supported(s->shape));
}

int effective_kernel(const ace_solver *s)
{
    int k = s->kernel;
    if (k == ACE_KERNEL_AUTO) k = s->tuned_kernel;
    if (k == ACE_KERNEL_AUTO) {
        if (s->p.total <= RESIDENT_MAX) k = ACE_KERNEL_RESIDENT;
        else if (s->p.d >= 2) k = ACE_KERNEL_TBLOCK;
        else k = ACE_KERNEL_DIRECT;
    }
    if (k == ACE_KERNEL_RESIDENT && s->p.total > RESIDENT_MAX) k = ACE_KERNEL_DIRECT;
    if (k == ACE_KERNEL_TBLOCK && !tblock_applies(s)) k = ACE_KERNEL_DIRECT;
    if (k == ACE_KERNEL_MARCH && !march_supported(s->shape)) k = ACE_KERNEL_DIRECT;
    return k;
}

// Steps one launch of `kernel` advances (in a long enough run).
// The register-resident 2D kernel is chosen and applies to the field.
bool use_tb2(const ace_solver *s) { return s->p.d == 2 && s->tb2 >= 0 && tb2_supported(s->shape); }

int steps_per_launch_of(const ace_solver *s, int kernel)
{
    if (kernel != ACE_KERNEL_TBLOCK) return 1;
    if (s->p.d == 3) return (s->tb3 >= 0 && tb3_supported(s->shape)) ? TB3_TABLE[s->tb3].depth : 2;
    return use_tb2(s) ? std::min(s->depth2, tb2_max_depth(s->tb2)) : s->depth2;
}

// One launch of the handle's 2D blocked kernel (K steps; level_stride > 0:
// every level written, as in launch_step_tblock2d).
hipError_t launch_blocked2d(const ace_solver *s, const double *in, double *out, double *parts,
                            int64_t *nparts, int K, int64_t level_stride, hipStream_t st)
{
    if (use_tb2(s)) return launch_step_tb2(s->tb2, s->shape, s->coef, in, out, parts, nparts, K, level_stride, st);
    return launch_step_tblock2d(s->shape, s->coef, in, out, parts, nparts, K, level_stride, st);
}

int64_t blocked2d_blocks(const ace_solver *s, int K)
{
    return use_tb2(s) ? tb2_blocks(s->tb2, s->shape, K) : tblock2d_blocks(s->shape, K);
}

bool use_tb3(const ace_solver *s, int kernel, int64_t remaining)
{
    return kernel == ACE_KERNEL_TBLOCK && s->p.d == 3 && s->tb3 >= 0 && tb3_supported(s->shape) &&
           remaining >= TB3_TABLE[s->tb3].depth;
}

// One launch from buf[cur] into buf[cur^1] advancing 1 step, or up to
// steps_per_launch_of() with the temporal-blocking kernels.  If want_mon,
// the monitor partials of the input field are left in s->partials, their
// count in *nparts.  Returns the number of steps taken (or a negative error).
// Partial triples a monitored launch of `kernel` writes (the launch that
// launch_steps makes for `remaining` steps).
int64_t partials_for(const ace_solver *s, int kernel, int64_t remaining)
{
    if (kernel == ACE_KERNEL_TBLOCK && s->p.d == 2)
        return blocked2d_blocks(s, (int)std::min<int64_t>(steps_per_launch_of(s, kernel), remaining));
    if (use_tb3(s, kernel, remaining)) return tb3_partials_needed(s->tb3, s->shape, s->zchunk);
    if (kernel == ACE_KERNEL_TBLOCK && remaining >= 2) return tblock_partials_needed(s->shape, s->zchunk);
    if (kernel == ACE_KERNEL_MARCH || kernel == ACE_KERNEL_TBLOCK) return march_partials_needed(s->shape);
    return direct_partials_needed(s->shape);
}

int launch_steps(ace_solver *s, int kernel, int64_t remaining, bool want_mon, int64_t *nparts)
{
    const double *in = s->buf[s->cur];
    double *out = s->buf[s->cur ^ 1];
    double *parts = want_mon ? s->partials : nullptr;
    if (want_mon && 3 * partials_for(s, kernel, remaining) > s->partials_cap) return ACE_E_STATE;
    hipError_t e;
    int taken = 1;
    if (kernel == ACE_KERNEL_TBLOCK && s->p.d == 2) {
        taken = (int)std::min<int64_t>(steps_per_launch_of(s, kernel), remaining);
        e = launch_blocked2d(s, in, out, parts, nparts, taken, 0, s->stream);
    } else if (use_tb3(s, kernel, remaining)) {
        e = launch_step_tb3(s->tb3, s->shape, s->coef, in, out, parts, nparts, s->zchunk, s->stream);
        taken = TB3_TABLE[s->tb3].depth;
    } else if (kernel == ACE_KERNEL_TBLOCK && remaining >= 2) {
        e = launch_step_tblock2(s->shape, s->coef, in, out, parts, nparts, s->zchunk, s->stream);
        taken = 2;
    } else if (kernel == ACE_KERNEL_MARCH || kernel == ACE_KERNEL_TBLOCK) {
        e = launch_step_march(s->shape, s->coef, in, out, parts, nparts, s->stream);
    } else {
        e = launch_step_direct(s->shape, s->coef, in, out, parts, nparts, s->stream);
    }
    ACE_HIP(e);
    s->cur ^= 1;
    s->steps += taken;
    return taken;
}

void drop_graphs(ace_solver *s)
{
    // a replay may still run on the handle's stream
    if (!s->graphs.empty()) (void)hipStreamSynchronize(s->stream);
    for (auto &g : s->graphs) {
        (void)hipGraphExecDestroy(g.e);
        (void)hipGraphDestroy(g.g);
    }
    s->graphs.clear();
}

// Graph of s->graph_launches launches (an even count, so the field returns to
// the same buffer) of `kernel` starting from buf[cur]; captured once on a
// private stream and replayed on the handle's stream.  Kernel nodes only.
int graph_for(ace_solver *s, int kernel, hipGraphExec_t *out)
{
    for (auto &g : s->graphs)
        if (g.kernel == kernel && g.zchunk == s->zchunk && g.depth2 == s->depth2 && g.tb3 == s->tb3 &&
            g.tb2 == s->tb2 && g.cur == s->cur &&
            g.b0 == s->buf[0] && g.b1 == s->buf[1]) {
            *out = g.e;
            return ACE_OK;
        }
    if (!s->capture) ACE_HIP(hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking));
    const hipStream_t user = s->stream;
    const int cur0 = s->cur;
    const int64_t steps0 = s->steps;
    s->stream = s->capture;
    ACE_HIP(hipStreamBeginCapture(s->capture, hipStreamCaptureModeThreadLocal));
    int rc = ACE_OK;
    const int per = steps_per_launch_of(s, kernel);
    for (int64_t i = 0; i < s->graph_launches && rc >= 0; ++i) {
        const int t = launch_steps(s, kernel, per, false, nullptr);
        if (t < 0) rc = t;
    }
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(s->capture, &g);
    s->stream = user;
    s->cur = cur0;
    s->steps = steps0;
    if (rc < 0) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    ACE_HIP(ce);
    hipGraphExec_t e = nullptr;
    hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_status(ie);
    }
    s->graphs.push_back({kernel, s->zchunk, s->depth2, s->tb3, s->tb2, cur0, s->buf[0], s->buf[1], g, e});
    if (log_enabled())
        fprintf(stderr,
                "[ace] graph: %lld launches of kernel %d, %d step(s) each (plane chunk %d, 2D depth %d, "
                "3D variant %d)\n",
                (long long)s->graph_launches, kernel, per, s->zchunk, s->depth2, s->tb3);
    *out = e;
    return ACE_OK;
}

int advance(ace_solver *s, int64_t nsteps)
{
    if (nsteps <= 0) return ACE_OK;
    const int k = effective_kernel(s);
    if (k == ACE_KERNEL_RESIDENT) {
        ACE_HIP(launch_resident(s->shape, s->coef, s->buf[s->cur], nsteps, 0, nullptr, s->stream));
        s->steps += nsteps;
        return ACE_OK;
    }
    const int per = steps_per_launch_of(s, k);
    int64_t i = 0;
    if (s->graph_launches >= 2) {
        const int64_t chunk = s->graph_launches * per;
        while (nsteps - i >= 2 * chunk) {
            hipGraphExec_t e = nullptr;
            ACE_TRY(graph_for(s, k, &e));
            ACE_HIP(hipGraphLaunch(e, s->stream));
            s->steps += chunk;  // even launch count: s->cur is unchanged
            i += chunk;
        }
    }
    while (i < nsteps) {
        const int t = launch_steps(s, k, nsteps - i, false, nullptr);
        if (t < 0) return t;
        i += t;
    }
    return ACE_OK;
}

int alloc_fields(ace_solver *s)
{
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipMalloc((void **)&s->own[i], (size_t)s->p.total * sizeof(double));
        if (e != hipSuccess) return hip_status(e);
        s->buf[i] = s->own[i];
    }
    // one partial triple per workgroup of any monitored launch
    int64_t need2 = 3 * std::max<int64_t>(
        std::max<int64_t>(monitor_partials_needed(s->shape), direct_partials_needed(s->shape)), 1);
    if (march_supported(s->shape)) need2 = std::max<int64_t>(need2, 3 * march_partials_needed(s->shape));
    if (tblock_supported(s->shape))
        need2 = std::max<int64_t>(need2, 3 * tblock_partials_needed(s->shape, TBLOCK_MIN_ZCHUNK));
    if (tb3_supported(s->shape))
        for (int v = 0; v < TB3_VARIANTS; ++v)
            need2 = std::max<int64_t>(need2, 3 * std::max<int64_t>(tb3_partials_needed(v, s->shape, 0),
                                                                 tb3_partials_needed(v, s->shape, TBLOCK_MIN_ZCHUNK)));
    if (tblock2d_supported(s->shape)) {
        need2 = std::max<int64_t>(need2, 3 * tblock2d_blocks(s->shape, tblock2d_max_depth()));
        if (tb2_supported(s->shape))
            for (int v = 0; v < TB2_VARIANTS; ++v)
                need2 = std::max<int64_t>(need2, 3 * tb2_blocks(v, s->shape, tb2_max_depth(v)));
    }
    ACE_TRY(grow(&s->partials, &s->partials_cap, need2));
    ACE_HIP(hipHostMalloc((void **)&s->pinned, 64 * sizeof(double), hipHostMallocDefault));
    return ACE_OK;
}

int read_triple(ace_solver *s, const double *dev, double *host3)
{
    ACE_HIP(hipMemcpyAsync(s->pinned, dev, 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    ACE_HIP(hipStreamSynchronize(s->stream));
    memcpy(host3, s->pinned, 3 * sizeof(double));
    return ACE_OK;
}

// Monitor triple of the current field into dev_out[0..2] (stream-ordered).
int monitor_now(ace_solver *s, double *dev_out)
{
    int64_t np = 0;
    if (3 * monitor_partials_needed(s->shape) > s->partials_cap) return ACE_E_STATE;
    ACE_HIP(launch_monitor(s->shape, s->buf[s->cur], s->partials, &np, s->stream));
    ACE_HIP(launch_reduce(s->partials, np, dev_out, s->stream));
    return ACE_OK;
}

// Autotuner cache: one JSON object per line and tuned problem shape,
//   {"d": 2, "bc": 0, "M": [1024, 1024, 1], "kernel": 4, "zchunk": 32,
//    "depth2": 5, "tb3": -1, "tb2": 0, "ms_per_step": 0.003389}
// appended by ace_autotune (kTuneFormat) and read back with the same format;
// the last matching line wins, other lines are skipped.
constexpr const char *kTuneFormat =
    "{\"d\": %d, \"bc\": %d, \"M\": [%lld, %lld, %lld], \"kernel\": %d, \"zchunk\": %d, "
    "\"depth2\": %d, \"tb3\": %d, \"tb2\": %d, \"ms_per_step\": %lf}";

void load_tuning(ace_solver *s)
{
    const char *path = getenv("ACE_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        int d, bc, k, zc, k2, v3, v2;
        long long m0, m1, m2;
        double ms;
        if (sscanf(line, kTuneFormat, &d, &bc, &m0, &m1, &m2, &k, &zc, &k2, &v3, &v2, &ms) != 11) continue;
        if (d == s->p.d && bc == s->p.bc && m0 == s->p.M[0] && m1 == s->p.M[1] && m2 == s->p.M[2] &&
            k >= ACE_KERNEL_DIRECT && k <= ACE_KERNEL_TBLOCK &&
            (zc == 0 || zc >= TBLOCK_MIN_ZCHUNK) && k2 >= 1 && k2 <= tblock2d_max_depth() && v3 >= -1 &&
            v3 < TB3_VARIANTS && v2 >= -1 && v2 < TB2_VARIANTS) {
            s->tuned_kernel = k;
            s->zchunk = zc;
            s->depth2 = k2;
            s->tb3 = v3;
            s->tb2 = v2;
        }
    }
    fclose(f);
}

}  // namespace

extern "C" {

const char *ace_version(void) { return "ace-mi355x 0.1 (gfx950, fp64)"; }

const char *ace_strerror(int st)
{
    switch (st) {
    case ACE_OK: return "ok";
    case ACE_E_ARG: return "invalid argument";
    case ACE_E_SIZE: return "too few cells for the boundary condition";
    case ACE_E_ANISO: return "grid spacing differs between axes";
    case ACE_E_DT: return "time step outside (0, 2): the cubic has no unique real root";
    case ACE_E_HIP: return "HIP runtime error";
    case ACE_E_NOMEM: return "out of memory";
    case ACE_E_NONFINITE: return "non-finite value in the field";
    case ACE_E_STATE: return "call not valid in the current state";
    case ACE_W_CONDITIONS: return "warning: dt > 1 - 2 d kappa (maximum-principle condition fails)";
    case ACE_W_PHI0_GT1: return "warning: |phi0| > 1 somewhere";
    case ACE_W_MAXPRINCIPLE: return "warning: max-norm exceeded 1 under the step condition";
    case ACE_W_ENERGY_UP: return "warning: energy increased under the step condition";
    default: return "unknown status";
    }
}

int ace_create(int d, const int64_t *N, const double *L, const double *R, double eps, double dt,
               int bc, ace_solver **out)
{
    if (!out) return ACE_E_ARG;
    *out = nullptr;
    Problem p;
    const int rc = derive(d, N, L, R, eps, dt, bc, p);
    if (rc < 0) return rc;
    ace_solver *s = new (std::nothrow) ace_solver();
    if (!s) return ACE_E_NOMEM;
    s->p = p;
    s->shape = shape_of(p);
    s->coef = coef_of(p);
    (void)hipGetDevice(&s->device);
    scratch_setup(s->device);
    const int arc = alloc_fields(s);
    if (arc < 0) {
        ace_destroy(s);
        return arc;
    }
    load_tuning(s);
    hipError_t e = hipMalloc((void **)&s->gsum, 4 * sizeof(double));
    if (e != hipSuccess) {
        ace_destroy(s);
        return hip_status(e);
    }
    if (log_enabled())
        fprintf(stderr, "[ace] create d=%d bc=%d M=%lldx%lldx%lld dx=%.6g kappa=%.6g h=%.6g Newton steps %d%s%s\n",
                p.d, p.bc, (long long)p.M[0], (long long)p.M[1], (long long)p.M[2], p.dx, p.kappa, p.h, p.nit,
                p.start2 ? " (second-order start)" : "", p.cond_ok ? "" : ", outside Theorem 2's conditions");
    *out = s;
    return rc;
}

int ace_destroy(ace_solver *s)
{
    if (!s) return ACE_E_ARG;
    drop_graphs(s);
    if (s->capture) (void)hipStreamDestroy(s->capture);
    if (s->aux) (void)hipStreamDestroy(s->aux);
    hipEvent_t evs[] = {s->ev_start, s->ev_rec[0], s->ev_rec[1], s->ev_rev[0], s->ev_rev[1]};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    for (int i = 0; i < 2; ++i)
        if (s->own[i]) (void)hipFree(s->own[i]);
    double *devs[] = {s->partials, s->mon, s->ckpt, s->seg, s->lam, s->gpart, s->gsum};
    for (double *p : devs)
        if (p) (void)hipFree(p);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
    return ACE_OK;
}

int ace_shape(const ace_solver *s, int64_t M[3], int64_t *total)
{
    if (!s) return ACE_E_ARG;
    if (M)
        for (int j = 0; j < 3; ++j) M[j] = s->p.M[j];
    if (total) *total = s->p.total;
    return ACE_OK;
}

int ace_node_coords(const ace_solver *s, int axis, double *x)
{
    if (!s || !x || axis < 0 || axis >= s->p.d) return ACE_E_ARG;
    const double L = s->p.L[axis], dx = s->p.dx;
    for (int64_t i = 0; i < s->p.M[axis]; ++i) {
        // Sec. 2: x_i = dx (i - 1/2) for HN, dx i for HD (i = 1..N-1) and P
        if (s->p.bc == ACE_BC_HN) x[i] = L + ((double)i - 0.5) * dx;
        else if (s->p.bc == ACE_BC_HD) x[i] = L + (double)(i + 1) * dx;
        else x[i] = L + (double)i * dx;
    }
    return ACE_OK;
}

int ace_params(const ace_solver *s, ace_params_t *q)
{
    if (!s || !q) return ACE_E_ARG;
    memset(q, 0, sizeof(*q));
    const Problem &p = s->p;
    q->d = p.d;
    q->bc = p.bc;
    for (int j = 0; j < 3; ++j) {
        q->N[j] = p.N[j];
        q->M[j] = p.M[j];
    }
    q->total = p.total;
    q->dx = p.dx;
    q->dt = p.dt;
    q->eps = p.eps;
    q->kappa = p.kappa;
    q->h = p.h;
    q->dt_bound = p.dx * p.dx / (p.dx * p.dx + 2.0 * p.d * p.eps * p.eps);
    // Sec. 4: omega_1 = 1/3, 1/5, 1/6 for d = 1, 2, 3; s = omega_1 / kappa
    q->omega1 = (p.d == 1) ? 1.0 / 3.0 : (p.d == 2 ? 0.2 : 1.0 / 6.0);
    q->s = q->omega1 / p.kappa;
    q->conditions_ok = p.cond_ok;
    q->newton_iters = p.nit;
    q->scheme = p.scheme;
    return ACE_OK;
}

int ace_set_stream(ace_solver *s, void *st)
{
    if (!s) return ACE_E_ARG;
    // a replay on the old stream may still use a captured graph
    if ((hipStream_t)st != s->stream) drop_graphs(s);
    s->stream = (hipStream_t)st;
    return ACE_OK;
}

int ace_bind_fields(ace_solver *s, double *a, double *b)
{
    if (!s) return ACE_E_ARG;
    if ((a == nullptr) != (b == nullptr) || (a && a == b)) return ACE_E_ARG;
    if (a) {
        s->buf[0] = a;
        s->buf[1] = b;
    } else {
        s->buf[0] = s->own[0];
        s->buf[1] = s->own[1];
    }
    s->cur = 0;
    s->steps = 0;
    s->field_version++;
    drop_graphs(s);
    return ACE_OK;
}

int ace_set_graph_launches(ace_solver *s, int64_t launches)
{
    if (!s || launches < 0) return ACE_E_ARG;
    s->graph_launches = launches + (launches & 1);  // even: the buffer parity returns
    drop_graphs(s);
    return ACE_OK;
}

int ace_set_eps(ace_solver *s, double eps)
{
    if (!s) return ACE_E_ARG;
    Problem q;
    int rc = derive(s->p.d, s->p.N, s->p.L, s->p.R, eps, s->p.dt, s->p.bc, q);
    if (rc < 0) return rc;
    q.scheme = s->p.scheme;
    set_conditions(q);
    rc = q.cond_ok ? ACE_OK : ACE_W_CONDITIONS;
    s->p = q;
    s->coef = coef_of(q);
    s->ck_count = 0;  // checkpoints of the old eps are no longer valid
    drop_graphs(s);   // captured launches carry the old coefficients
    return rc;
}

int ace_set_scheme(ace_solver *s, int scheme)
{
    if (!s || (scheme != ACE_SCHEME_RLB_MIE && scheme != ACE_SCHEME_FEX)) return ACE_E_ARG;
    s->p.scheme = scheme;
    set_conditions(s->p);
    s->coef = coef_of(s->p);
    s->ck_count = 0;
    drop_graphs(s);
    return s->p.cond_ok ? ACE_OK : ACE_W_CONDITIONS;
}

int ace_set_kernel(ace_solver *s, int kernel, int depth)
{
    if (!s || kernel < ACE_KERNEL_AUTO || kernel > ACE_KERNEL_TBLOCK || depth < 0) return ACE_E_ARG;
    if (kernel == ACE_KERNEL_TBLOCK && depth != 0) {
        if (s->p.d == 3 && (depth < 2 || depth > 4)) return ACE_E_ARG;
        if (s->p.d == 2 && depth > tblock2d_max_depth()) return ACE_E_ARG;
        if (s->p.d == 2) s->depth2 = depth;
        if (s->p.d == 3) s->tb3 = (depth == 2) ? -1 : (depth == 3 ? TB3_DEFAULT_DEPTH3 : TB3_DEFAULT_DEPTH4);
    }
    s->kernel = kernel;
    s->depth = depth;
    return ACE_OK;
}

int ace_set_region3d(ace_solver *s, int depth, int rows, int rows_per_thread)
{
    if (!s || s->p.d != 3) return ACE_E_ARG;
    if (depth == 2 && rows == 0 && rows_per_thread == 0) {
        s->tb3 = -1;
        return ACE_OK;
    }
    const int v = tb3_find(depth, rows, rows_per_thread);
    if (v < 0) return ACE_E_ARG;
    s->tb3 = v;
    return ACE_OK;
}

int ace_get_region3d(const ace_solver *s, int *depth, int *rows, int *rows_per_thread)
{
    if (!s || !depth || !rows || !rows_per_thread || s->p.d != 3) return ACE_E_ARG;
    if (s->tb3 < 0) {
        *depth = 2;
        *rows = 0;
        *rows_per_thread = 0;
    } else {
        *depth = TB3_TABLE[s->tb3].depth;
        *rows = TB3_TABLE[s->tb3].rows;
        *rows_per_thread = TB3_TABLE[s->tb3].rpt;
    }
    return ACE_OK;
}

int ace_set_region2d(ace_solver *s, int rows, int rows_per_thread)
{
    if (!s || s->p.d != 2) return ACE_E_ARG;
    if (rows == 0 && rows_per_thread == 0) {
        s->tb2 = -1;
        return ACE_OK;
    }
    const int v = tb2_find(rows, rows_per_thread);
    if (v < 0) return ACE_E_ARG;
    s->tb2 = v;
    return ACE_OK;
}

int ace_get_region2d(const ace_solver *s, int *rows, int *rows_per_thread)
{
    if (!s || !rows || !rows_per_thread || s->p.d != 2) return ACE_E_ARG;
    *rows = s->tb2 >= 0 ? TB2_TABLE[s->tb2].rows : 0;
    *rows_per_thread = s->tb2 >= 0 ? TB2_TABLE[s->tb2].rpt : 0;
    return ACE_OK;
}

int ace_set_plane_chunk(ace_solver *s, int planes)
{
    if (!s || s->p.d != 3 || (planes != 0 && (planes < TBLOCK_MIN_ZCHUNK || planes > 4096)))
        return ACE_E_ARG;
    s->zchunk = planes;
    return ACE_OK;
}

int ace_get_plane_chunk(const ace_solver *s, int *planes)
{
    if (!s || !planes) return ACE_E_ARG;
    *planes = s->zchunk;
    return ACE_OK;
}

int ace_get_kernel(const ace_solver *s, int *kernel, int *steps_per_launch)
{
    if (!s || !kernel) return ACE_E_ARG;
    const int k = effective_kernel(s);
    *kernel = k;
    if (steps_per_launch) *steps_per_launch = steps_per_launch_of(s, k);
    return ACE_OK;
}

int ace_set_phi0(ace_solver *s, const double *phi0, int where)
{
    if (!s || !phi0 || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    int warn = ACE_OK;
    const size_t bytes = (size_t)s->p.total * sizeof(double);
    if (where == ACE_HOST) {
        for (int64_t i = 0; i < s->p.total; ++i) {
            if (!isfinite(phi0[i])) return ACE_E_NONFINITE;
            if (fabs(phi0[i]) > 1.0) warn = ACE_W_PHI0_GT1;
        }
        ACE_HIP(hipMemcpyAsync(s->buf[0], phi0, bytes, hipMemcpyHostToDevice, s->stream));
        ACE_HIP(hipStreamSynchronize(s->stream));
    } else {
        ACE_HIP(hipMemcpyAsync(s->buf[0], phi0, bytes, hipMemcpyDeviceToDevice, s->stream));
    }
    s->cur = 0;
    s->steps = 0;
    s->field_version++;
    return warn;
}

int ace_step(ace_solver *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return ACE_E_ARG;
    ACE_TRY(advance(s, nsteps));
    s->field_version++;
    return ACE_OK;
}

int ace_run_monitored(ace_solver *s, int64_t nsteps, int64_t every, double *E, double *maxn)
{
    if (!s || nsteps < 0 || every < 1 || !E || !maxn) return ACE_E_ARG;
    const int64_t nmon = nsteps / every + 1;
    ACE_TRY(grow(&s->mon, &s->mon_cap, 3 * nmon));
    const int k = effective_kernel(s);
    if (k == ACE_KERNEL_RESIDENT) {
        ACE_HIP(launch_resident(s->shape, s->coef, s->buf[s->cur], nsteps, every, s->mon, s->stream));
        s->steps += nsteps;
    } else {
        int64_t j = 0;
        for (int64_t st = 0; st <= nsteps; st += every) {
            if (st == nsteps) {
                ACE_TRY(monitor_now(s, s->mon + 3 * j));
            } else {
                const int64_t seg = std::min<int64_t>(every, nsteps - st);
                int64_t np = 0;
                int64_t done = launch_steps(s, k, seg, true, &np);
                if (done < 0) return (int)done;
                ACE_HIP(launch_reduce(s->partials, np, s->mon + 3 * j, s->stream));
                while (done < seg) {
                    const int t = launch_steps(s, k, seg - done, false, nullptr);
                    if (t < 0) return t;
                    done += t;
                }
            }
            ++j;
        }
    }
    s->field_version++;
    std::vector<double> trip((size_t)(3 * nmon));
    ACE_HIP(hipMemcpyAsync(trip.data(), s->mon, trip.size() * sizeof(double), hipMemcpyDeviceToHost,
                           s->stream));
    ACE_HIP(hipStreamSynchronize(s->stream));
    for (int64_t j = 0; j < nmon; ++j) {
        E[j] = energy_from(s->p, &trip[3 * j]);
        maxn[j] = trip[3 * j + 2];
    }
    return ace_monitor_status(nmon, E, maxn, s->p.cond_ok, &s->warn_mask);
}

int ace_get_warnings(const ace_solver *s, int *mask)
{
    if (!s || !mask) return ACE_E_ARG;
    *mask = s->warn_mask;
    return ACE_OK;
}

int ace_monitor_status(int64_t n, const double *E, const double *maxn, int conditions_ok, int *mask)
{
    if (mask) *mask = 0;
    if (n < 1 || !E || !maxn) return ACE_E_ARG;
    int bits = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (!isfinite(maxn[j]) || !isfinite(E[j])) return ACE_E_NONFINITE;
        if (!conditions_ok) continue;
        // Theorem 2: |phi| <= 1 is kept; Theorem 3: the energy does not rise
        if (maxn[j] > 1.0 + 4.0 * 0x1p-53) bits |= ACE_WARN_BIT(ACE_W_MAXPRINCIPLE);
        if (j > 0 && E[j] > E[j - 1] + 1e-14 * fabs(E[j - 1])) bits |= ACE_WARN_BIT(ACE_W_ENERGY_UP);
    }
    if (mask) *mask = bits;
    if (bits & ACE_WARN_BIT(ACE_W_MAXPRINCIPLE)) return ACE_W_MAXPRINCIPLE;
    if (bits & ACE_WARN_BIT(ACE_W_ENERGY_UP)) return ACE_W_ENERGY_UP;
    return ACE_OK;
}

int ace_energy(ace_solver *s, double *E)
{
    if (!s || !E) return ACE_E_ARG;
    ACE_TRY(grow(&s->mon, &s->mon_cap, 3));
    ACE_TRY(monitor_now(s, s->mon));
    double t[3];
    ACE_TRY(read_triple(s, s->mon, t));
    *E = energy_from(s->p, t);
    return isfinite(*E) ? ACE_OK : ACE_E_NONFINITE;
}

int ace_maxnorm(ace_solver *s, double *m)
{
    if (!s || !m) return ACE_E_ARG;
    ACE_TRY(grow(&s->mon, &s->mon_cap, 3));
    ACE_TRY(monitor_now(s, s->mon));
    double t[3];
    ACE_TRY(read_triple(s, s->mon, t));
    *m = t[2];
    return isfinite(*m) ? ACE_OK : ACE_E_NONFINITE;
}

int ace_phase_volume(ace_solver *s, double *V)
{
    if (!s || !V) return ACE_E_ARG;
    ACE_TRY(grow(&s->partials, &s->partials_cap, phase_partials_needed()));
    ACE_TRY(grow(&s->mon, &s->mon_cap, 3));
    ACE_HIP(launch_phase_volume(s->buf[s->cur], s->p.total, s->partials, s->mon, s->stream));
    double t[3];
    ACE_TRY(read_triple(s, s->mon, t));
    *V = pow(s->p.dx, s->p.d) * t[0];
    return isfinite(*V) ? ACE_OK : ACE_E_NONFINITE;
}

int ace_monitor_noalloc(ace_solver *s, const double *phi, double *out)
{
    if (!s || !out) return ACE_E_ARG;
    double *scr = scratch_of(s->device);
    if (!scr) return ACE_E_STATE;
    const int64_t np = monitor_partials_needed(s->shape);
    if (np < 1 || np > kNoAllocParts) return ACE_E_SIZE;
    const double *f = phi ? phi : s->buf[s->cur];
    int64_t n2 = 0;
    ACE_HIP(launch_monitor(s->shape, f, scr + kTripSlot, &n2, s->stream));
    ACE_HIP(launch_reduce(scr + kTripSlot, n2, scr, s->stream));
    double dxd, cg;
    energy_coefs(s->p, &dxd, &cg);
    ACE_HIP(launch_monitor_finish(scr, dxd, cg, out, s->stream));
    return ACE_OK;
}

int ace_equivalent_radius(ace_solver *s, double *R)
{
    if (!s || !R) return ACE_E_ARG;
    double V = 0.0;
    ACE_TRY(ace_phase_volume(s, &V));
    // Sec. 4.2.2: the circle (V = pi R^2) and the sphere (V = 4/3 pi R^3);
    // in 1D the phase is an interval of length 2R
    if (s->p.d == 1) *R = 0.5 * V;
    else if (s->p.d == 2) *R = sqrt(V / M_PI);
    else *R = cbrt(3.0 * V / (4.0 * M_PI));
    return isfinite(*R) ? ACE_OK : ACE_E_NONFINITE;
}

int ace_get_phi(ace_solver *s, double *out, int where)
{
    if (!s || !out || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    const size_t bytes = (size_t)s->p.total * sizeof(double);
    ACE_HIP(hipMemcpyAsync(out, s->buf[s->cur], bytes,
                           where == ACE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           s->stream));
    if (where == ACE_HOST) ACE_HIP(hipStreamSynchronize(s->stream));
    return ACE_OK;
}

int64_t ace_step_count(const ace_solver *s) { return s ? s->steps : -1; }

const double *ace_field_ptr(const ace_solver *s) { return s ? s->buf[s->cur] : nullptr; }

// Shortest timed trial of the autotuner, and the most steps a lengthened
// trial may take.
constexpr double kMinTrialMs = 2.0;
constexpr int64_t kMaxTrialSteps = 1 << 20;

int ace_autotune(ace_solver *s, int64_t trial_steps, char *json, size_t cap)
{
    if (!s || trial_steps < 1) return ACE_E_ARG;
    struct Cand {
        int kernel, zchunk, depth2, tb3, tb2;
    };
    std::vector<Cand> cands;
    const int z0c = s->zchunk, k0 = s->depth2, v30 = s->tb3, v20 = s->tb2;
    cands.push_back({ACE_KERNEL_DIRECT, z0c, k0, v30, v20});
    if (s->p.total <= RESIDENT_MAX) cands.push_back({ACE_KERNEL_RESIDENT, z0c, k0, v30, v20});
    if (march_supported(s->shape)) cands.push_back({ACE_KERNEL_MARCH, z0c, k0, v30, v20});
    if (s->p.d == 3 && tblock_supported(s->shape))
        for (int zc : {0, 16, 24, 32, 40, 48, 64, 128})  // 0: persistent grid
            if (zc <= std::max<int64_t>(s->shape.M0, 16)) cands.push_back({ACE_KERNEL_TBLOCK, zc, k0, -1, v20});
    // the configurable 3D kernel: every depth and region shape, fewer plane
    // chunks.  Long chunks matter when a chunk count leaves the last round of
    // one-workgroup-per-CU launches half empty (512^3 at depth 3: 117 tiles x
    // 8 chunks of 64 = 936 workgroups on 256 CUs, against 234 of 256 planes).
    if (s->p.d == 3 && tb3_supported(s->shape))
        for (int v = 0; v < TB3_VARIANTS; ++v)
            for (int zc : {0, 16, 32, 64, 128, 256})
                if (zc <= std::max<int64_t>(s->shape.M0, 16)) cands.push_back({ACE_KERNEL_TBLOCK, zc, k0, v, v20});
    if (s->p.d == 2 && tblock2d_supported(s->shape)) {
        for (int k2 : {1, 2, 3, 4, 5, 6, 8, 10, 12})
            if (k2 <= tblock2d_max_depth()) cands.push_back({ACE_KERNEL_TBLOCK, z0c, k2, v30, -1});
        // the register-resident 2D kernel: every region shape and depth
        for (int v = 0; v < (tb2_supported(s->shape) ? TB2_VARIANTS : 0); ++v)
            for (int k2 : {2, 3, 4, 5, 6, 8, 10, 12})
                if (k2 <= tb2_max_depth(v)) cands.push_back({ACE_KERNEL_TBLOCK, z0c, k2, v30, v});
    }
    const int64_t total = s->p.total;
    double *save = nullptr;
    ACE_HIP(hipMalloc((void **)&save, sizeof(double) * total));
    const int cur0 = s->cur;
    const int64_t steps0 = s->steps;
    const int kernel0 = s->kernel, zchunk0 = s->zchunk, depth20 = s->depth2, tb30 = s->tb3, tb20 = s->tb2;
    int rc = hip_status(hipMemcpyAsync(save, s->buf[cur0], sizeof(double) * total,
                                       hipMemcpyDeviceToDevice, s->stream));
    auto restore = [&]() {
        s->cur = cur0;
        return hip_status(hipMemcpyAsync(s->buf[cur0], save, sizeof(double) * total,
                                         hipMemcpyDeviceToDevice, s->stream));
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc >= 0) rc = hip_status(hipEventCreate(&e0));
    if (rc >= 0) rc = hip_status(hipEventCreate(&e1));
    // restores the field, then times `n` steps on the handle's stream
    auto time_run = [&](int64_t n, float *out) -> int {
        int r;
        if ((r = restore()) < 0) return r;
        if ((r = hip_status(hipEventRecord(e0, s->stream))) < 0) return r;
        if ((r = advance(s, n)) < 0) return r;
        if ((r = hip_status(hipEventRecord(e1, s->stream))) < 0) return r;
        if ((r = hip_status(hipEventSynchronize(e1))) < 0) return r;
        return hip_status(hipEventElapsedTime(out, e0, e1));
    };
    std::string rec = "{\"kind\": \"solver\", \"trial_steps\": " + std::to_string(trial_steps) +
                      ", \"candidates\": [";
    double best_ms = 1e300;
    Cand best = cands[0];
    bool first = true;
    for (const Cand &c : cands) {
        if (rc < 0) break;
        s->kernel = c.kernel;
        s->zchunk = c.zchunk;
        s->depth2 = c.depth2;
        s->tb3 = c.tb3;
        s->tb2 = c.tb2;
        // Each length is run once untimed (code object load, graph capture)
        // and then timed.  A trial shorter than kMinTrialMs is lengthened to
        // about that, so small fields are timed in the steady state of a long
        // run (graph replay) rather than on a few directly issued launches.
        int64_t steps = trial_steps;
        float ms = 0.f;
        if ((rc = time_run(steps, &ms)) < 0) break;
        if ((rc = time_run(steps, &ms)) < 0) break;
        if (ms < kMinTrialMs && steps < kMaxTrialSteps) {
            const double scale = kMinTrialMs / std::max<double>(ms, 1e-3);
            steps = std::min<int64_t>(kMaxTrialSteps, (int64_t)ceil((double)steps * scale));
            if ((rc = time_run(steps, &ms)) < 0) break;
            if ((rc = time_run(steps, &ms)) < 0) break;
        }
        const double per = ms / (double)steps;
        char buf[320];
        const int d3 = c.tb3 >= 0 ? TB3_TABLE[c.tb3].depth : 2;
        const int r3 = c.tb3 >= 0 ? TB3_TABLE[c.tb3].rows : 0, t3 = c.tb3 >= 0 ? TB3_TABLE[c.tb3].rpt : 0;
        const int r2 = c.tb2 >= 0 ? TB2_TABLE[c.tb2].rows : 0, t2 = c.tb2 >= 0 ? TB2_TABLE[c.tb2].rpt : 0;
        snprintf(buf, sizeof buf,
                 "%s{\"kernel\": %d, \"zchunk\": %d, \"depth2\": %d, \"tb3\": %d, \"depth3\": %d, "
                 "\"rows\": %d, \"rows_per_thread\": %d, \"tb2\": %d, \"rows2\": %d, "
                 "\"rows_per_thread2\": %d, \"steps\": %lld, \"ms_per_step\": %.6f}",
                 first ? "" : ", ", c.kernel, c.zchunk, c.depth2, c.tb3, d3, r3, t3, c.tb2, r2, t2, (long long)steps,
                 per);
        rec += buf;
        first = false;
        if (per < best_ms) {
            best_ms = per;
            best = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    s->kernel = kernel0;
    s->zchunk = zchunk0;
    s->depth2 = depth20;
    s->tb3 = tb30;
    s->tb2 = tb20;
    if (rc >= 0) rc = restore();
    if (rc >= 0) rc = hip_status(hipStreamSynchronize(s->stream));
    (void)hipFree(save);
    s->steps = steps0;
    if (rc < 0) return rc;
    s->tuned_kernel = best.kernel;
    s->zchunk = best.zchunk;
    s->depth2 = best.depth2;
    s->tb3 = best.tb3;
    s->tb2 = best.tb2;
    drop_graphs(s);
    char buf[320];
    {
        const int d3 = best.tb3 >= 0 ? TB3_TABLE[best.tb3].depth : 2;
        const int r3 = best.tb3 >= 0 ? TB3_TABLE[best.tb3].rows : 0;
        const int t3 = best.tb3 >= 0 ? TB3_TABLE[best.tb3].rpt : 0;
        const int r2 = best.tb2 >= 0 ? TB2_TABLE[best.tb2].rows : 0;
        const int t2 = best.tb2 >= 0 ? TB2_TABLE[best.tb2].rpt : 0;
        snprintf(buf, sizeof buf,
                 "], \"choice\": {\"kernel\": %d, \"zchunk\": %d, \"depth2\": %d, \"tb3\": %d, "
                 "\"depth3\": %d, \"rows\": %d, \"rows_per_thread\": %d, \"tb2\": %d, \"rows2\": %d, "
                 "\"rows_per_thread2\": %d, \"ms_per_step\": %.6f}}",
                 best.kernel, best.zchunk, best.depth2, best.tb3, d3, r3, t3, best.tb2, r2, t2, best_ms);
    }
    rec += buf;
    if (json && cap > 0) snprintf(json, cap, "%s", rec.c_str());
    if (log_enabled())
        fprintf(stderr,
                "[ace] autotune d=%d bc=%d M=%lldx%lldx%lld: kernel %d, plane chunk %d, 2D depth %d, "
                "3D variant %d, 2D variant %d, %.6f ms/step\n",
                s->p.d, s->p.bc, (long long)s->p.M[0], (long long)s->p.M[1], (long long)s->p.M[2], best.kernel,
                best.zchunk, best.depth2, best.tb3, best.tb2, best_ms);
    const char *path = getenv("ACE_AUTOTUNE_CACHE");
    if (path) {
        FILE *f = fopen(path, "a");
        if (f) {
            // the same fields as kTuneFormat, ms written with a fixed precision
            fprintf(f,
                    "{\"d\": %d, \"bc\": %d, \"M\": [%lld, %lld, %lld], \"kernel\": %d, \"zchunk\": %d, "
                    "\"depth2\": %d, \"tb3\": %d, \"tb2\": %d, \"ms_per_step\": %.6f}\n",
                    s->p.d, s->p.bc, (long long)s->p.M[0], (long long)s->p.M[1], (long long)s->p.M[2],
                    best.kernel, best.zchunk, best.depth2, best.tb3, best.tb2, best_ms);
            fclose(f);
        }
    }
    return ACE_OK;
}

// ---------------------------------------------------------------------------
// reverse mode
// ---------------------------------------------------------------------------

int ace_forward_ckpt(ace_solver *s, const double *phi0, int where, int64_t nsteps, int64_t every)
{
    if (!s || !phi0 || nsteps < 0 || every < 1) return ACE_E_ARG;
    if (s->p.scheme != ACE_SCHEME_RLB_MIE) return ACE_E_STATE;
    const int rc = ace_set_phi0(s, phi0, where);
    if (rc < 0) return rc;
    const int64_t total = s->p.total;
    const int64_t nck = nsteps == 0 ? 1 : (nsteps + every - 1) / every;
    ACE_TRY(grow(&s->ckpt, &s->ckpt_cap, nck * total));
    // size the reverse sweep's buffers now so ace_backward allocates nothing
    ACE_TRY(grow(&s->seg, &s->seg_cap, 2 * (every + 1) * total));
    ACE_TRY(grow(&s->lam, &s->lam_cap, 2 * total));
    int64_t per_step = adjoint_partials_needed(s->shape);
    if (tblock2d_supported(s->shape))
        per_step = std::max<int64_t>(per_step, tblock2d_blocks(s->shape, tblock2d_max_depth()));
    ACE_TRY(grow(&s->gpart, &s->gpart_cap, per_step * every));
    const size_t bytes = (size_t)total * sizeof(double);
    for (int64_t j = 0; j < nck; ++j) {
        ACE_HIP(hipMemcpyAsync(s->ckpt + j * total, s->buf[s->cur], bytes, hipMemcpyDeviceToDevice,
                               s->stream));
        const int64_t n = std::min<int64_t>(every, nsteps - j * every);
        ACE_TRY(advance(s, n));
    }
    s->field_version++;
    s->ck_every = every;
    s->ck_steps = nsteps;
    s->ck_count = nck;
    s->ck_field_version = s->field_version;
    s->ck_generation++;
    return rc;
}

int64_t ace_ckpt_generation(const ace_solver *s) { return s ? s->ck_generation : -1; }

int ace_backward(ace_solver *s, const double *lambdaT, double *dphi0, double *deps2, int where)
{
    if (!s || !lambdaT || !dphi0 || !deps2 || (where != ACE_HOST && where != ACE_DEVICE))
        return ACE_E_ARG;
    if (s->ck_count <= 0 || s->ck_field_version != s->field_version) return ACE_E_STATE;
    const int64_t total = s->p.total, every = s->ck_every, nsteps = s->ck_steps;
    const size_t bytes = (size_t)total * sizeof(double);
    if (s->seg_cap < 2 * (every + 1) * total || s->lam_cap < 2 * total) return ACE_E_STATE;
    const int64_t npart = adjoint_partials_needed(s->shape);
    double *lam[2] = {s->lam, s->lam + total};
    int lc = 0;
    // The reverse sweep of segment j (on the handle's stream) and the
    // recompute of segment j-1 (on a second stream) are independent, so they
    // run concurrently on alternating segment buffers; events order each
    // buffer's recompute after the previous sweep that used it, and each sweep
    // after its recompute.
    if (!s->aux) ACE_HIP(hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking));
    if (!s->ev_start) {
        ACE_HIP(hipEventCreateWithFlags(&s->ev_start, hipEventDisableTiming));
        for (int b = 0; b < 2; ++b) {
            ACE_HIP(hipEventCreateWithFlags(&s->ev_rec[b], hipEventDisableTiming));
            ACE_HIP(hipEventCreateWithFlags(&s->ev_rev[b], hipEventDisableTiming));
        }
    }
    ACE_HIP(hipMemcpyAsync(lam[0], lambdaT, bytes,
                           where == ACE_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                           s->stream));
    ACE_HIP(hipMemsetAsync(s->gsum, 0, sizeof(double), s->stream));
    ACE_HIP(hipEventRecord(s->ev_start, s->stream));  // checkpoints are complete
    ACE_HIP(hipStreamWaitEvent(s->aux, s->ev_start, 0));
    int k = effective_kernel(s);
    if (k == ACE_KERNEL_RESIDENT) k = ACE_KERNEL_DIRECT;
    const bool blocked2d = (k == ACE_KERNEL_TBLOCK && s->p.d == 2);
    if (k == ACE_KERNEL_TBLOCK && !blocked2d) k = ACE_KERNEL_MARCH;
    for (int64_t j = s->ck_count - 1; j >= 0; --j) {
        const int b = (int)(j & 1);
        double *seg = s->seg + b * (every + 1) * total;
        const int64_t a = j * every;
        const int64_t n = std::min<int64_t>(every, nsteps - a);
        // --- recompute segment j on the second stream ---
        ACE_HIP(hipStreamWaitEvent(s->aux, s->ev_rev[b], 0));
        ACE_HIP(hipMemcpyAsync(seg, s->ckpt + j * total, bytes, hipMemcpyDeviceToDevice, s->aux));
        if (blocked2d) {
            const int per = steps_per_launch_of(s, ACE_KERNEL_TBLOCK);
            for (int64_t i = 0; i < n;) {  // each launch writes its K intermediate states
                const int K = (int)std::min<int64_t>(per, n - i);
                ACE_HIP(launch_blocked2d(s, seg + i * total, seg + (i + 1) * total, nullptr, nullptr, K, total,
                                         s->aux));
                i += K;
            }
        } else {
            for (int64_t i = 0; i < n; ++i) {
                const double *in = seg + i * total;
                double *out = seg + (i + 1) * total;
                hipError_t e = (k == ACE_KERNEL_MARCH)
                                   ? launch_step_march(s->shape, s->coef, in, out, nullptr, nullptr, s->aux)
                                   : launch_step_direct(s->shape, s->coef, in, out, nullptr, nullptr, s->aux);
                ACE_HIP(e);
            }
        }
        ACE_HIP(hipEventRecord(s->ev_rec[b], s->aux));
        // --- reverse sweep of segment j on the handle's stream ---
        ACE_HIP(hipStreamWaitEvent(s->stream, s->ev_rec[b], 0));
        int64_t parts = 0;  // partial sums of dL/dkappa written for this segment
        if (blocked2d) {
            const int64_t nb = tblock2d_blocks(s->shape, s->depth2);
            for (int64_t i = n; i > 0;) {  // K transposed steps per launch
                const int K = (int)std::min<int64_t>(s->depth2, i);
                ACE_HIP(launch_adjoint_tblock2d(s->shape, s->coef, lam[lc], seg + (i - K) * total, total,
                                                lam[lc ^ 1], s->gpart + parts, K, s->stream));
                parts += (K == s->depth2) ? nb : tblock2d_blocks(s->shape, K);
                lc ^= 1;
                i -= K;
            }
        } else {
            for (int64_t i = n - 1; i >= 0; --i) {
                ACE_HIP(launch_adjoint_step(s->shape, s->coef, lam[lc], seg + i * total,
                                            seg + (i + 1) * total, lam[lc ^ 1], s->gpart + parts,
                                            nullptr, s->stream));
                parts += npart;
                lc ^= 1;
            }
        }
        if (parts > 0) ACE_HIP(launch_sum(s->gpart, parts, s->gsum, 1, s->stream));
        ACE_HIP(hipEventRecord(s->ev_rev[b], s->stream));
    }
    ACE_HIP(hipMemcpyAsync(dphi0, lam[lc], bytes,
                           where == ACE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                           s->stream));
    ACE_HIP(hipMemcpyAsync(s->pinned, s->gsum, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    ACE_HIP(hipStreamSynchronize(s->stream));
    // kappa = eps^2 dt / dx^2  =>  dL/d(eps^2) = (dt / dx^2) dL/dkappa
    *deps2 = s->pinned[0] * s->p.dt / (s->p.dx * s->p.dx);
    return ACE_OK;
}

int ace_adjoint(ace_solver *s, const double *phi0, int64_t nsteps, int64_t ckpt_every,
                const double *lambdaT, double *dphi0, double *deps2, int where)
{
    const int rc = ace_forward_ckpt(s, phi0, where, nsteps, ckpt_every);
    if (rc < 0) return rc;
    return ace_backward(s, lambdaT, dphi0, deps2, where);
}

}  // extern "C"
