// Step kernels that need no tiling: one thread per node (any d, any BC),
// the LDS-resident multi-step kernel for small fields, the standalone
// monitor pass, and the fixed-order reductions.
#include "ace_device.h"

namespace ace {

namespace {

constexpr int kBlock = 256;

// Neighbour sum and monitor terms of node (i0, i1, i2) read through the
// cache.  Axis order of the sum: the paper's axes from the slowest to the
// fastest stored index.
template <int D, int BC, bool MON>
__device__ __forceinline__ double node_update(const Shape &s, const StepCoef &c,
                                              const double *__restrict__ in,
                                              int64_t i0, int64_t i1, int64_t i2,
                                              MonAcc &m)
{
    const int64_t idx = (i0 * s.M1 + i1) * s.M2 + i2;
    const double p = in[idx];
    double nsum = 0.0;
    double grad = 0.0;
    const int64_t coord[3] = {i0, i1, i2};
    const int64_t size[3] = {s.M0, s.M1, s.M2};
    const int64_t stride[3] = {s.M1 * s.M2, s.M2, 1};
#pragma unroll
    for (int a = 3 - D; a < 3; ++a) {
        const int64_t cc = coord[a], n = size[a], st = stride[a];
        double lo, hi;
        if (cc > 0) lo = in[idx - st];
        else lo = outside<BC>(p, BC == BC_P ? in[idx + (n - 1) * st] : 0.0);
        if (cc < n - 1) hi = in[idx + st];
        else hi = outside<BC>(p, BC == BC_P ? in[idx - (n - 1) * st] : 0.0);
        nsum += lo + hi;
        if (MON) {
            const double dh = hi - p;
            grad = fma(dh, dh, grad);
            if (BC == BC_HD && cc == 0) grad = fma(p, p, grad);
        }
    }
    if (MON) {
        m.bulk += bulk_term(p);
        m.grad += grad;
        m.mx = nan_max(m.mx, fabs(p));
    }
    return update<D>(p, nsum, c);
}

template <int D, int BC, bool MON>
__global__ __launch_bounds__(kBlock) void k_step_direct(Shape s, StepCoef c,
                                                        const double *__restrict__ in,
                                                        double *__restrict__ out,
                                                        double *__restrict__ partials)
{
    __shared__ double lds[3 * (kBlock / 64)];
    const int64_t i2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i1 = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
    const int64_t i0 = blockIdx.z;
    MonAcc m;
    mon_zero(m);
    if (i2 < s.M2 && i1 < s.M1) {
        const double v = node_update<D, BC, MON>(s, c, in, i0, i1, i2, m);
        out[(i0 * s.M1 + i1) * s.M2 + i2] = v;
    }
    if (MON) {
        const int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
        block_reduce_store(m, lds, partials + 3 * b);
    }
}

template <int D, int BC>
__global__ __launch_bounds__(kBlock) void k_monitor(Shape s, const double *__restrict__ in,
                                                    double *__restrict__ partials)
{
    __shared__ double lds[3 * (kBlock / 64)];
    const int64_t i2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i1 = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
    const int64_t i0 = blockIdx.z;
    MonAcc m;
    mon_zero(m);
    if (i2 < s.M2 && i1 < s.M1) {
        const int64_t idx = (i0 * s.M1 + i1) * s.M2 + i2;
        const double p = in[idx];
        const int64_t coord[3] = {i0, i1, i2};
        const int64_t size[3] = {s.M0, s.M1, s.M2};
        const int64_t stride[3] = {s.M1 * s.M2, s.M2, 1};
        double grad = 0.0;
#pragma unroll
        for (int a = 3 - D; a < 3; ++a) {
            const int64_t cc = coord[a], n = size[a], st = stride[a];
            double hi;
            if (cc < n - 1) hi = in[idx + st];
            else hi = outside<BC>(p, BC == BC_P ? in[idx - (n - 1) * st] : 0.0);
            const double dh = hi - p;
            grad = fma(dh, dh, grad);
            if (BC == BC_HD && cc == 0) grad = fma(p, p, grad);
        }
        m.bulk = bulk_term(p);
        m.grad = grad;
        m.mx = fabs(p);
    }
    const int64_t b = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
    block_reduce_store(m, lds, partials + 3 * b);
}

void direct_grid(const Shape &s, dim3 &grid, dim3 &block)
{
    int bx = 1;
    while (bx < s.M2 && bx < kBlock) bx <<= 1;
    if (s.d == 1) bx = kBlock;
    const int by = kBlock / bx;
    block = dim3(bx, by, 1);
    grid = dim3((unsigned)((s.M2 + bx - 1) / bx), (unsigned)((s.M1 + by - 1) / by), (unsigned)s.M0);
}

template <bool MON>
hipError_t dispatch_direct(const Shape &s, const StepCoef &c, const double *in, double *out,
                           double *partials, dim3 grid, dim3 block, hipStream_t st)
{
#define ACE_DIRECT(DD, BB)                                                                 \
    if (s.d == DD && s.bc == BB) {                                                         \
        hipLaunchKernelGGL((k_step_direct<DD, BB, MON>), grid, block, 0, st, s, c, in, out, \
                           partials);                                                      \
        return hipGetLastError();                                                          \
    }
    ACE_DIRECT(1, BC_HN) ACE_DIRECT(1, BC_HD) ACE_DIRECT(1, BC_P)
    ACE_DIRECT(2, BC_HN) ACE_DIRECT(2, BC_HD) ACE_DIRECT(2, BC_P)
    ACE_DIRECT(3, BC_HN) ACE_DIRECT(3, BC_HD) ACE_DIRECT(3, BC_P)
#undef ACE_DIRECT
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Whole field resident in LDS.  One workgroup; each thread owns up to
// kResNodes nodes and keeps their neighbours' LDS slots in registers.  Slot
// `total` always holds 0.0 and stands for the Dirichlet wall.
// ---------------------------------------------------------------------------
constexpr int kResThreads = 1024;
constexpr int kResNodes = (int)((RESIDENT_MAX + kResThreads - 1) / kResThreads);

// The field alternates between two LDS buffers (one barrier per step); RV
// is the root variant of update_n (0: start and Newton count at run time).
template <int D, int BC, int RV>
__global__ __launch_bounds__(kResThreads) void k_resident(Shape s, StepCoef c,
                                                          double *__restrict__ field,
                                                          int64_t nsteps, int64_t every,
                                                          double *__restrict__ mon)
{
    __shared__ double fb[2][RESIDENT_MAX + 1];
    __shared__ double red[3 * (kResThreads / 64)];
    const int total = (int)(s.M0 * s.M1 * s.M2);
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int M[3] = {(int)s.M0, (int)s.M1, (int)s.M2};
    const int str[3] = {(int)(s.M1 * s.M2), (int)s.M2, 1};
    int nb_lo[kResNodes][3], nb_hi[kResNodes][3];
#pragma unroll
    for (int k = 0; k < kResNodes; ++k) {
        const int j = tid + k * nt;
        int rem = j < total ? j : 0;
        const int cc[3] = {rem / str[0], (rem / str[1]) % M[1], rem % M[2]};
#pragma unroll
        for (int a = 3 - D; a < 3; ++a) {
            const int n = M[a], st = str[a];
            int lo, hi;
            if (cc[a] > 0) lo = j - st;
            else lo = (BC == BC_HN) ? j : (BC == BC_HD ? total : j + (n - 1) * st);
            if (cc[a] < n - 1) hi = j + st;
            else hi = (BC == BC_HN) ? j : (BC == BC_HD ? total : j - (n - 1) * st);
            nb_lo[k][a] = lo;
            nb_hi[k][a] = hi;
        }
    }
    for (int j = tid; j < total; j += nt) fb[0][j] = field[j];
    if (tid == 0) {
        fb[0][total] = 0.0;
        fb[1][total] = 0.0;
    }
    __syncthreads();
    int64_t jm = 0;
    int cb = 0;
    for (int64_t step = 0;; ++step) {
        const double *f = fb[cb];
        if (every > 0 && step % every == 0) {
            MonAcc m;
            mon_zero(m);
#pragma unroll
            for (int k = 0; k < kResNodes; ++k) {
                const int j = tid + k * nt;
                if (j < total) {
                    const double p = f[j];
                    double g = 0.0;
#pragma unroll
                    for (int a = 3 - D; a < 3; ++a) {
                        const double dh = f[nb_hi[k][a]] - p;
                        g = fma(dh, dh, g);
                        if (BC == BC_HD && nb_lo[k][a] == total) g = fma(p, p, g);
                    }
                    m.bulk += bulk_term(p);
                    m.grad += g;
                    m.mx = nan_max(m.mx, fabs(p));
                }
            }
            block_reduce_store(m, red, mon + 3 * jm);
            ++jm;
            __syncthreads();
        }
        if (step == nsteps) break;
        double *fn = fb[cb ^ 1];
#pragma unroll
        for (int k = 0; k < kResNodes; ++k) {
            const int j = tid + k * nt;
            if (j < total) {
                const double p = f[j];
                double nsum = 0.0;
#pragma unroll
                for (int a = 3 - D; a < 3; ++a) nsum += f[nb_lo[k][a]] + f[nb_hi[k][a]];
                fn[j] = update_n<D, RV>(p, nsum, c);
            }
        }
        cb ^= 1;
        __syncthreads();
    }
    for (int j = tid; j < total; j += nt) field[j] = fb[cb][j];
}

__global__ __launch_bounds__(1024) void k_reduce(const double *__restrict__ partials, int64_t n,
                                                 double *__restrict__ out)
{
    __shared__ double lds[3 * 16];
    MonAcc m;
    mon_zero(m);
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        m.bulk += partials[3 * j + 0];
        m.grad += partials[3 * j + 1];
        m.mx = nan_max(m.mx, partials[3 * j + 2]);
    }
    block_reduce_store(m, lds, out);
}

// Per-block partial sums of (1 + phi)/2 (the smooth phase indicator), each
// block over a contiguous range in a fixed order: every thread keeps
// kPhaseU running sums over loads kPhaseU * 256 apart (so kPhaseU loads are
// in flight per thread), added in order at the end.
constexpr int kPhaseBlocks = 4096;
constexpr int kPhaseU = 8;
__global__ __launch_bounds__(256) void k_phase_partials(const double *__restrict__ f, int64_t n,
                                                        double *__restrict__ part)
{
    __shared__ double lds[4];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = (lo + per < n) ? lo + per : n;
    double acc[kPhaseU];
#pragma unroll
    for (int u = 0; u < kPhaseU; ++u) acc[u] = 0.0;
    int64_t j = lo + threadIdx.x;
    for (; j + (kPhaseU - 1) * 256 < hi; j += kPhaseU * 256) {
#pragma unroll
        for (int u = 0; u < kPhaseU; ++u) acc[u] += 0.5 * (1.0 + f[j + u * 256]);
    }
    for (; j < hi; j += 256) acc[0] += 0.5 * (1.0 + f[j]);
    double v = acc[0];
#pragma unroll
    for (int u = 1; u < kPhaseU; ++u) v += acc[u];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((lds[0] + lds[1]) + (lds[2] + lds[3]));
}

__global__ __launch_bounds__(1024) void k_sum(const double *__restrict__ x, int64_t n,
                                              double *__restrict__ out, int accumulate)
{
    __shared__ double lds[16];
    double v = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) v += x[j];
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += lds[k];
        out[0] = accumulate ? out[0] + t : t;
    }
}

}  // namespace

hipError_t launch_step_direct(const Shape &s, const StepCoef &c, const double *in, double *out,
                              double *partials, int64_t *nparts, hipStream_t st)
{
    dim3 grid, block;
    direct_grid(s, grid, block);
    if (nparts) *nparts = (int64_t)grid.x * grid.y * grid.z;
    if (partials) return dispatch_direct<true>(s, c, in, out, partials, grid, block, st);
    return dispatch_direct<false>(s, c, in, out, nullptr, grid, block, st);
}

// ---------------------------------------------------------------------------
// Monitor partials of a 2D/3D field on tiles marching along axis 0: a
// 256-thread workgroup owns 16 rows x 64 columns of the two fastest axes and
// a chunk of MZ planes, so the grid (and the partials the one-block
// reduction then reads) is small.  The per-node terms are those of k_monitor
// in the same order.  Each node is loaded once: one wavefront holds 64
// consecutive columns of MRY rows, the +x neighbour comes from the next lane
// (the column after the tile from one extra load, by lanes 0..MRY-1), the
// +y neighbour from the thread's next row (the row after its MRY rows from
// one extra load), the +z neighbour from the next plane.  Loads for plane
// z + 2 are issued while plane z is summed.  Past the field's end the extra
// loads read wrapped or clamped (always valid) coordinates, so every load is
// unconditional; HN and HD then replace the value as the BC requires.
// ---------------------------------------------------------------------------
constexpr int MTX = 64;  // one wavefront across the columns of a tile
constexpr int MTR = 4;
constexpr int MRY = 4;
constexpr int MTY = MTR * MRY;  // 16 rows per tile
constexpr int MNT = MTX * MTR;  // 256 threads
constexpr int MZ = 32;

template <int D, int BC>
__global__ __launch_bounds__(MNT) void k_monitor_tiles(Shape s, const double *__restrict__ in,
                                                      double *__restrict__ partials, int tiles_x,
                                                      int tiles_y)
{
    static_assert(MTX == 64, "the +x neighbour is taken from the next lane of the wavefront");
    __shared__ double lds[3 * (MNT / 64)];
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t ntile = (int64_t)tiles_x * tiles_y;
    const int tile = (int)(t % ntile);
    const int64_t chunk = t / ntile;
    const int lane = threadIdx.x & (MTX - 1);
    const int tr = threadIdx.x / MTX;
    const int64_t x0 = (int64_t)(tile % tiles_x) * MTX;
    const int64_t x = x0 + lane;
    const int64_t ybase = (int64_t)(tile / tiles_x) * MTY + tr * MRY;
    const int64_t PS = s.M1 * s.M2;
    const bool xin = x < s.M2;
    const int64_t cx = xin ? x : s.M2 - 1;
    const bool xlast = x + 1 >= s.M2;
    const bool x_from_edge = xlast || lane == MTX - 1;
    // column after the tile and row after the thread's rows (wrapped past the end)
    const int64_t xe = (x0 + MTX < s.M2) ? x0 + MTX : 0;
    const int64_t ye = ((ybase + MRY < s.M1) ? ybase + MRY : 0) * s.M2;
    int64_t row[MRY];
    bool yin[MRY], ylast[MRY];
#pragma unroll
    for (int r = 0; r < MRY; ++r) {
        const int64_t y = ybase + r;
        yin[r] = y < s.M1;
        ylast[r] = y + 1 >= s.M1;
        row[r] = (yin[r] ? y : s.M1 - 1) * s.M2;
    }
    // lane r < MRY loads the edge column of row r
    const int er = lane < MRY ? lane : MRY - 1;
    const int64_t eoff = (ybase + er < s.M1 ? ybase + er : s.M1 - 1) * s.M2 + xe;
    auto zmap = [&](int64_t zz) -> int64_t {  // plane index past the end: wrapped, then clamped
        if (zz < s.M0) return zz;
        zz -= s.M0;
        return zz < s.M0 ? zz : s.M0 - 1;
    };
    const int64_t z0 = chunk * MZ;
    const int64_t z1 = (z0 + MZ < s.M0) ? z0 + MZ : s.M0;
    MonAcc m;
    mon_zero(m);
    double cur[MRY], nxt[MRY], cye, cxe, nye = 0.0, nxe = 0.0;
    {
        const int64_t zb = z0 * PS;
#pragma unroll
        for (int r = 0; r < MRY; ++r) cur[r] = in[zb + row[r] + cx];
        cye = in[zb + ye + cx];
        cxe = in[zb + eoff];
        if (D == 3) {
            const int64_t zn = zmap(z0 + 1) * PS;
#pragma unroll
            for (int r = 0; r < MRY; ++r) nxt[r] = in[zn + row[r] + cx];
            nye = in[zn + ye + cx];
            nxe = in[zn + eoff];
        }
    }
    for (int64_t z = z0; z < z1; ++z) {
        double nn[MRY], nnye = 0.0, nnxe = 0.0;
        if (D == 3) {
            const int64_t z2 = zmap(z + 2) * PS;
#pragma unroll
            for (int r = 0; r < MRY; ++r) nn[r] = in[z2 + row[r] + cx];
            nnye = in[z2 + ye + cx];
            nnxe = in[z2 + eoff];
        }
        const bool zlast = z + 1 >= s.M0;
#pragma unroll
        for (int r = 0; r < MRY; ++r) {
            const double p = cur[r];
            const double from_lane = __shfl_down(p, 1, 64);
            const double from_edge = __shfl(cxe, r, 64);
            const double vx = x_from_edge ? from_edge : from_lane;
            const double vy = (ylast[r] || r == MRY - 1) ? cye : cur[r + 1 < MRY ? r + 1 : r];
            if (!(xin && yin[r])) continue;
            double grad = 0.0;
            if (D == 3) {
                const double hi = zlast ? outside<BC>(p, nxt[r]) : nxt[r];
                const double dh = hi - p;
                grad = fma(dh, dh, grad);
                if (BC == BC_HD && z == 0) grad = fma(p, p, grad);
            }
            {
                const double hi = ylast[r] ? outside<BC>(p, vy) : vy;
                const double dh = hi - p;
                grad = fma(dh, dh, grad);
                if (BC == BC_HD && ybase + r == 0) grad = fma(p, p, grad);
            }
            {
                const double hi = xlast ? outside<BC>(p, vx) : vx;
                const double dh = hi - p;
                grad = fma(dh, dh, grad);
                if (BC == BC_HD && x == 0) grad = fma(p, p, grad);
            }
            m.bulk += bulk_term(p);
            m.grad += grad;
            m.mx = nan_max(m.mx, fabs(p));
        }
        if (D == 3) {
#pragma unroll
            for (int r = 0; r < MRY; ++r) {
                cur[r] = nxt[r];
                nxt[r] = nn[r];
            }
            cye = nye;
            cxe = nxe;
            nye = nnye;
            nxe = nnxe;
        }
    }
    block_reduce_store(m, lds, partials + 3 * blockIdx.x);
}

void monitor_tiles_grid(const Shape &s, int &tiles_x, int &tiles_y, int64_t &nblk)
{
    tiles_x = (int)((s.M2 + MTX - 1) / MTX);
    tiles_y = (int)((s.M1 + MTY - 1) / MTY);
    nblk = (int64_t)tiles_x * tiles_y * ((s.M0 + MZ - 1) / MZ);
}

int64_t direct_partials_needed(const Shape &s)
{
    dim3 grid, block;
    direct_grid(s, grid, block);
    return (int64_t)grid.x * grid.y * grid.z;
}

int64_t monitor_partials_needed(const Shape &s)
{
    if (s.d == 1) {
        dim3 grid, block;
        direct_grid(s, grid, block);
        return (int64_t)grid.x * grid.y * grid.z;
    }
    int tx, ty;
    int64_t nblk;
    monitor_tiles_grid(s, tx, ty, nblk);
    return nblk;
}

hipError_t launch_monitor(const Shape &s, const double *in, double *partials, int64_t *nparts,
                          hipStream_t st)
{
    if (s.d == 1) {
        dim3 grid, block;
        direct_grid(s, grid, block);
        if (nparts) *nparts = (int64_t)grid.x * grid.y * grid.z;
        switch (s.bc) {
        case BC_HN: hipLaunchKernelGGL((k_monitor<1, BC_HN>), grid, block, 0, st, s, in, partials); break;
        case BC_HD: hipLaunchKernelGGL((k_monitor<1, BC_HD>), grid, block, 0, st, s, in, partials); break;
        case BC_P: hipLaunchKernelGGL((k_monitor<1, BC_P>), grid, block, 0, st, s, in, partials); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    int tx, ty;
    int64_t nblk;
    monitor_tiles_grid(s, tx, ty, nblk);
    if (nparts) *nparts = nblk;
#define ACE_MON(DD, BB)                                                                              \
    if (s.d == DD && s.bc == BB) {                                                                   \
        hipLaunchKernelGGL((k_monitor_tiles<DD, BB>), dim3((unsigned)nblk), dim3(MNT), 0, st, s, in, \
                           partials, tx, ty);                                                        \
        return hipGetLastError();                                                                    \
    }
    ACE_MON(2, BC_HN) ACE_MON(2, BC_HD) ACE_MON(2, BC_P)
    ACE_MON(3, BC_HN) ACE_MON(3, BC_HD) ACE_MON(3, BC_P)
#undef ACE_MON
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(const double *partials, int64_t nparts, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partials, nparts, out);
    return hipGetLastError();
}

// E = dxd (bulk + cg grad) and the max-norm of a reduced monitor triple, on
// the device (the same operations, in the same order, as the host's
// energy_from, so both give the same bits).
__global__ void k_monitor_finish(const double *__restrict__ trip, double dxd, double cg,
                                 double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = dxd * (trip[0] + cg * trip[1]);
        out[1] = trip[2];
    }
}

hipError_t launch_monitor_finish(const double *trip, double dxd, double cg, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_monitor_finish, dim3(1), dim3(64), 0, st, trip, dxd, cg, out);
    return hipGetLastError();
}

int64_t phase_partials_needed() { return kPhaseBlocks; }

hipError_t launch_phase_volume(const double *f, int64_t n, double *part, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_phase_partials, dim3(kPhaseBlocks), dim3(256), 0, st, f, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, part, (int64_t)kPhaseBlocks, out, 0);
    return hipGetLastError();
}

hipError_t launch_sum(const double *x, int64_t n, double *out, int accumulate, hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, x, n, out, accumulate);
    return hipGetLastError();
}

hipError_t launch_resident(const Shape &s, const StepCoef &c, double *field, int64_t nsteps,
                           int64_t every, double *mon, hipStream_t st)
{
    const int64_t total = s.M0 * s.M1 * s.M2;
    if (total > RESIDENT_MAX || total < 1) return hipErrorInvalidValue;
    int threads = (int)((total + 63) / 64 * 64);
    if (threads > kResThreads) threads = kResThreads;
    // every node index tid + k * threads must fit in kResNodes slots
    if ((total + threads - 1) / threads > kResNodes) return hipErrorInvalidValue;
#define ACE_RES_N(DD, BB, NN)                                                                    \
    hipLaunchKernelGGL((k_resident<DD, BB, NN>), dim3(1), dim3(threads), 0, st, s, c, field, nsteps, \
                       every, mon);                                                              \
    return hipGetLastError();
#define ACE_RES(DD, BB)                          \
    if (s.d == DD && s.bc == BB) {               \
        switch (root_variant(c)) {               \
        case 1: { ACE_RES_N(DD, BB, 1) }         \
        case 2: { ACE_RES_N(DD, BB, 2) }         \
        case 3: { ACE_RES_N(DD, BB, 3) }         \
        case 5: { ACE_RES_N(DD, BB, 5) }         \
        case 6: { ACE_RES_N(DD, BB, 6) }         \
        default: { ACE_RES_N(DD, BB, 0) }        \
        }                                        \
    }
    ACE_RES(1, BC_HN) ACE_RES(1, BC_HD) ACE_RES(1, BC_P)
    ACE_RES(2, BC_HN) ACE_RES(2, BC_HD) ACE_RES(2, BC_P)
    ACE_RES(3, BC_HN) ACE_RES(3, BC_HD) ACE_RES(3, BC_P)
#undef ACE_RES
#undef ACE_RES_N
    return hipErrorInvalidValue;
}

}  // namespace ace
