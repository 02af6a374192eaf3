// Mesoscopic form of the scheme (Sec. 2): the 2d+1 populations of the
// DdQ(2d+1) lattice under the regularized evolution equation, before the
// summation over k that yields the macroscopic FD step.
//
// Per node, with phi = sum_k f_k of the populations at the node and at its
// 2d neighbours (out-of-range neighbours take the boundary condition's
// value), the right-hand sides are
//   R_0     = w_0 (phi - h f(phi))
//   R_{+a}  = w_1 (phi_{-a} - h f(phi)) - A (phi - phi_{-a})   (from x - e_a)
//   R_{-a}  = w_1 (phi_{+a} - h f(phi)) + A (phi_{+a} - phi)   (from x + e_a)
// with A = w_1 (1 - s)/s: the equilibrium w_k phi of the upwind node, the
// regularized non-equilibrium part s_A w_k c_k . Pi^ne with
// Pi^ne = -dt c_s^2 grad(phi)/s and the first-order gradient between the
// upwind node and x (c dt = dx, so c_s^2 and c cancel), and the source half
// (dt/2) F_k at t.  The summed left-hand side is theta + h f(theta), so the
// new phi is the root theta of the same cubic as the FD step, and
// f_k(t + dt) = R_k - w_k h f(theta).
//
// Populations are stored one array per k (k = 0 at rest, 1..d along +axis,
// d+1..2d along -axis, axis 0 the slowest), each `ps` doubles apart (the
// node count rounded up to 32 plus a 1280-byte stagger, so every array
// starts on 256 bytes and the arrays do not start on the same HBM channel).
// Any step reads each node's 2d+1 populations and writes them: at least
// 16 (2d+1) bytes of HBM per node update, against 16 for the FD step.
// The new populations depend on the old ones only through phi.  Four launch
// forms compute the same result bit for bit: one thread per node
// (k_pop_direct); a tiled march on cache-line-aligned tiles that sums phi
// from the populations itself (k_pop_update, fused: 16 (2d+1) bytes per node
// update); the split form, a streaming moment pass (k_pop_moment) then the
// same tiled update reading phi (16 (2d+1) + 16 bytes); and the carried
// form, in which each update also writes phi of its new populations (summed
// in the same order as every moment here, so it equals a moment pass bit
// for bit) and the next update reads only that (8 (2d+1) + 16 bytes).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/ace.h"
#include "ace_device.h"
#include "ace_runtime.h"

namespace ace {

namespace {

struct PopCoef {
    StepCoef sc;  // root of the cubic (h, omh, h3, nit)
    double w0, w1;
    double A;     // w_1 (1 - s)/s
    int64_t ps;   // stride between population arrays
};

// New populations of one node from phi at the node (p) and at its
// neighbours lo[a] = phi(x - e_a), hi[a] = phi(x + e_a), a = 0..D-1.
template <int D, int RV>
__device__ __forceinline__ void pop_update(double p, const double (&lo)[D], const double (&hi)[D],
                                           const PopCoef &c, double (&out)[2 * D + 1])
{
    const double hf = c.sc.h * fma(p, p * p, -p);
    double r[2 * D + 1];
    r[0] = c.w0 * (p - hf);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        r[1 + a] = fma(c.w1, lo[a] - hf, -c.A * (p - lo[a]));
        r[1 + D + a] = fma(c.w1, hi[a] - hf, c.A * (hi[a] - p));
    }
    double xi = r[0];
#pragma unroll
    for (int k = 1; k < 2 * D + 1; ++k) xi += r[k];
    const double th = cubic_root_n<RV>(xi, c.sc);
    const double hft = c.sc.h * fma(th, th * th, -th);
    out[0] = fma(-c.w0, hft, r[0]);
#pragma unroll
    for (int k = 1; k < 2 * D + 1; ++k) out[k] = fma(-c.w1, hft, r[k]);
}

// Zeroth moment at flat node i: sum_k f_k, k = 0..2D in order (every kernel
// sums in this order, so all of them see the same phi).
template <int D>
__device__ __forceinline__ double phi_at(const double *__restrict__ f, int64_t ps, int64_t i)
{
    double v = f[i];
#pragma unroll
    for (int k = 1; k < 2 * D + 1; ++k) v += f[k * ps + i];
    return v;
}

// Coordinate mapped into [0, n) (always a valid address).  Out-of-range
// coordinates follow the boundary condition: Neumann clamps (the neighbour
// of a wall node is the node itself), periodic wraps, Dirichlet clamps and
// sets `zero` (the value there is 0).
template <int BC>
__device__ __forceinline__ int64_t pmap(int64_t c, int64_t n, bool &zero)
{
    if (c >= 0 && c < n) return c;
    if (BC == BC_P) {
        int64_t m = c % n;
        return m < 0 ? m + n : m;
    }
    if (BC == BC_HD) zero = true;
    return c < 0 ? 0 : n - 1;
}

// ---- one thread per node (any d; the reference the tiled kernel matches) --
template <int D, int BC, int RV>
__global__ __launch_bounds__(256) void k_pop_direct(Shape s, PopCoef c, const double *__restrict__ fin,
                                                    double *__restrict__ fout)
{
    const int64_t n = s.M0 * s.M1 * s.M2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t M[3] = {s.M0, s.M1, s.M2};
    const int64_t st[3] = {s.M1 * s.M2, s.M2, 1};
    const int64_t co[3] = {i / st[0], (i / st[1]) % s.M1, i % s.M2};
    const double p = phi_at<D>(fin, c.ps, i);
    double lo[D], hi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int ax = 3 - D + a;  // the d axes are the last d of the three
        bool zl = false, zh = false;
        const int64_t cl = pmap<BC>(co[ax] - 1, M[ax], zl);
        const int64_t ch = pmap<BC>(co[ax] + 1, M[ax], zh);
        const double vl = phi_at<D>(fin, c.ps, i + (cl - co[ax]) * st[ax]);
        const double vh = phi_at<D>(fin, c.ps, i + (ch - co[ax]) * st[ax]);
        lo[a] = zl ? 0.0 : vl;
        hi[a] = zh ? 0.0 : vh;
    }
    double out[2 * D + 1];
    pop_update<D, RV>(p, lo, hi, c, out);
#pragma unroll
    for (int k = 0; k < 2 * D + 1; ++k) fout[k * c.ps + i] = out[k];
}

// s_waitcnt immediate of vmcnt(0) alone (gfx9 encoding: vmcnt bits 3:0 and
// 15:14 zero, expcnt 6:4 and lgkmcnt 11:8 at their maxima)
constexpr int VMCNT0 = 0x0F70;

// ---- tiled update (d = 2, 3) ------------------------------------------------
// Writes the new populations from phi (the split form, phi written by
// k_pop_moment) or straight from the populations (fused).  A workgroup owns
// a UOY x UX output tile aligned to whole cache lines (each wavefront stores
// 64 consecutive doubles of every population array; each thread URYT rows of
// one column); phi of the tile plus its one-node ring sits in LDS, ring node
// h loaded by thread h % UNT (URPT extra loads per thread; a thread past the
// ring's end loads its own node again, so every load is unconditional).  In 3D the
// workgroup marches along axis 0 with phi of planes z-1, z, z+1 of its own
// nodes in registers.  The default tile is 16 x 128 on 512 threads (4 rows
// per thread): against 16 x 64 it halves the ring columns per node, whose
// lines are fetched for one value each (1.375 lines per tile line instead of
// 1.625), which with 128-plane chunks made the 3D step 11% faster.
template <int X, int TR, int RYT>
struct PopTile {
    static constexpr int UX = X;                      // columns (a power of two, >= 64)
    static constexpr int UTR = TR;                    // thread rows
    static constexpr int URYT = RYT;                  // rows per thread
    static constexpr int UOY = UTR * URYT;            // rows of the tile
    static constexpr int ULW = UX + 2;                // LDS plane with its one-node ring
    static constexpr int ULH = UOY + 2;
    static constexpr int ULP = ULW * ULH;
    static constexpr int UNT = UX * UTR;              // threads
    static constexpr int URING = 2 * UX + 2 * UOY;    // ring nodes
    static constexpr int URPT = (URING + UNT - 1) / UNT;  // ring nodes per thread
    static_assert((UX & (UX - 1)) == 0 && UX >= 64, "tile columns: a power of two, whole wavefronts");
};
using PopTileDefault = PopTile<128, 4, 4>;  // 16 x 128, 512 threads

// FUSED: `src` holds the populations and phi of every node the tile needs is
// summed here from its 2d+1 arrays (k = 0..2d in order, as everywhere);
// otherwise `src` is phi (written by k_pop_moment or carried).  CARRY: phi of
// the new populations (k = 0..2d in order) also goes to phi_out.
template <class T, int D, int BC, int RV, bool FUSED, bool CARRY>
__global__ __launch_bounds__(T::UNT) void k_pop_update(Shape s, PopCoef c, const double *__restrict__ src,
                                                       double *__restrict__ fout, double *__restrict__ phi_out,
                                                       int tiles_x, int tiles_y, int zchunk)
{
    constexpr int UX = T::UX, URYT = T::URYT, UOY = T::UOY, ULW = T::ULW, ULH = T::ULH,
                  ULP = T::ULP, URING = T::URING, URPT = T::URPT, UNT = T::UNT;
    constexpr int Q = 2 * D + 1;
    constexpr int QIN = FUSED ? Q : 1;
    __shared__ double L[2 * ULP];
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t ntile = (int64_t)tiles_x * tiles_y;
    const int tile = (int)(t % ntile);
    const int64_t chunk = t / ntile;
    const int64_t x0 = (int64_t)(tile % tiles_x) * UX, y0 = (int64_t)(tile / tiles_x) * UOY;
    const int lx = threadIdx.x & (UX - 1);
    const int tr = threadIdx.x / UX;
    const int64_t PS = s.M1 * s.M2;

    // own nodes
    int64_t off[URYT], oidx[URYT];
    bool zr[URYT], ok[URYT];
    const int64_t xg = x0 + lx;
    bool zx = false;
    const int64_t mx = pmap<BC>(xg, s.M2, zx);
#pragma unroll
    for (int r = 0; r < URYT; ++r) {
        const int64_t yg = y0 + tr * URYT + r;
        bool zy = false;
        const int64_t my = pmap<BC>(yg, s.M1, zy);
        off[r] = my * s.M2 + mx;
        zr[r] = zx || zy;
        ok[r] = xg < s.M2 && yg < s.M1;
        oidx[r] = ok[r] ? yg * s.M2 + xg : 0;
    }
    // ring slots of this thread: ring node threadIdx.x + j * UNT for
    // j < URPT (a thread past the ring's end reloads its own first node)
    int hslot[URPT];
    int64_t hoff[URPT];
    bool hz[URPT];
#pragma unroll
    for (int j = 0; j < URPT; ++j) {
        const int h = threadIdx.x + j * UNT;
        hslot[j] = -1;
        hoff[j] = off[0];
        hz[j] = zr[0];
        if (h < URING) {
            int64_t hy, hx;
            int ly, lxx;
            if (h < UX) {  // row above
                hy = y0 - 1; hx = x0 + h; ly = 0; lxx = 1 + h;
            } else if (h < 2 * UX) {  // row below
                hy = y0 + UOY; hx = x0 + (h - UX); ly = ULH - 1; lxx = 1 + (h - UX);
            } else if (h < 2 * UX + UOY) {  // column left
                hy = y0 + (h - 2 * UX); hx = x0 - 1; ly = 1 + (h - 2 * UX); lxx = 0;
            } else {  // column right
                hy = y0 + (h - 2 * UX - UOY); hx = x0 + UX; ly = 1 + (h - 2 * UX - UOY); lxx = ULW - 1;
            }
            bool z1 = false, z2 = false;
            const int64_t my = pmap<BC>(hy, s.M1, z1);
            const int64_t mxx = pmap<BC>(hx, s.M2, z2);
            hoff[j] = my * s.M2 + mxx;
            hz[j] = z1 || z2;
            hslot[j] = ly * ULW + lxx;
        }
    }

    double own_raw[QIN][URYT], ring_raw[QIN][URPT];
    bool zown = false, zring = false;
    auto issue_own = [&](int64_t zz) {
        zown = false;
        const int64_t base = pmap<BC>(zz, s.M0, zown) * PS;
#pragma unroll
        for (int r = 0; r < URYT; ++r)
#pragma unroll
            for (int k = 0; k < QIN; ++k) own_raw[k][r] = src[k * c.ps + base + off[r]];
    };
    auto issue_ring = [&](int64_t zz) {
        zring = false;
        const int64_t base = pmap<BC>(zz, s.M0, zring) * PS;
#pragma unroll
        for (int j = 0; j < URPT; ++j)
#pragma unroll
            for (int k = 0; k < QIN; ++k) ring_raw[k][j] = src[k * c.ps + base + hoff[j]];
    };
    auto own_val = [&](int r) {
        double v = own_raw[0][r];
#pragma unroll
        for (int k = 1; k < QIN; ++k) v += own_raw[k][r];
        return (zown || zr[r]) ? 0.0 : v;
    };
    auto stage = [&](double *Lb, const double (&pc)[URYT]) {
#pragma unroll
        for (int r = 0; r < URYT; ++r) Lb[(1 + tr * URYT + r) * ULW + 1 + lx] = pc[r];
#pragma unroll
        for (int j = 0; j < URPT; ++j) {
            double v = ring_raw[0][j];
#pragma unroll
            for (int k = 1; k < QIN; ++k) v += ring_raw[k][j];
            if (hslot[j] >= 0) Lb[hslot[j]] = (zring || hz[j]) ? 0.0 : v;
        }
    };
    double outv[URYT][Q];
    auto update_plane = [&](const double *Lc, const double (&pm)[URYT], const double (&pc)[URYT],
                            const double (&pp)[URYT]) {
#pragma unroll
        for (int r = 0; r < URYT; ++r) {
            if (!ok[r]) continue;
            const int ly = 1 + tr * URYT + r, lxx = 1 + lx;
            const double p = pc[r];
            const double xm = Lc[ly * ULW + lxx - 1], xp = Lc[ly * ULW + lxx + 1];
            // y neighbours: the thread's own rows from registers, the rows
            // beyond them from LDS
            const double ym = (r == 0) ? Lc[(ly - 1) * ULW + lxx] : pc[r > 0 ? r - 1 : 0];
            const double yp = (r == URYT - 1) ? Lc[(ly + 1) * ULW + lxx] : pc[r + 1 < URYT ? r + 1 : r];
            if constexpr (D == 3) {
                const double lo[3] = {pm[r], ym, xm}, hi[3] = {pp[r], yp, xp};
                pop_update<3, RV>(p, lo, hi, c, outv[r]);
            } else {
                const double lo[2] = {ym, xm}, hi[2] = {yp, xp};
                pop_update<2, RV>(p, lo, hi, c, outv[r]);
            }
        }
    };
    auto store_plane = [&](int64_t z) {
#pragma unroll
        for (int r = 0; r < URYT; ++r) {
            if (!ok[r]) continue;
            const int64_t o = z * PS + oidx[r];
            // the new populations are not read again by this launch:
            // streaming (non-temporal) stores keep them out of the way of the
            // inputs in L2
#pragma unroll
            for (int k = 0; k < Q; ++k) __builtin_nontemporal_store(outv[r][k], fout + k * c.ps + o);
            if (CARRY) {
                // the zeroth moment of the new populations, in the order of phi_at
                double v = outv[r][0];
#pragma unroll
                for (int k = 1; k < Q; ++k) v += outv[r][k];
                phi_out[o] = v;
            }
        }
    };

    if constexpr (D == 2) {
        double pc[URYT];
        issue_own(0);
        issue_ring(0);
#pragma unroll
        for (int r = 0; r < URYT; ++r) pc[r] = own_val(r);
        stage(L, pc);
        __syncthreads();
        update_plane(L, pc, pc, pc);
        store_plane(0);
    } else {
        const int64_t z0 = chunk * zchunk;
        const int64_t z1 = std::min<int64_t>(z0 + zchunk, s.M0);
        double pm[URYT], pc[URYT], pp[URYT];
        issue_own(z0 - 1);
#pragma unroll
        for (int r = 0; r < URYT; ++r) pm[r] = own_val(r);
        issue_own(z0);
#pragma unroll
        for (int r = 0; r < URYT; ++r) pc[r] = own_val(r);
        issue_ring(z0);
        stage(L, pc);
        issue_own(z0 + 1);
#pragma unroll
        for (int r = 0; r < URYT; ++r) pp[r] = own_val(r);
        int b = 0;
        __syncthreads();
        for (int64_t z = z0; z < z1; ++z) {
            // own nodes of plane z+2 and the ring of plane z+1 (past the
            // chunk the loads repeat a valid plane, unused)
            issue_own(z + 2 < z1 + 1 ? z + 2 : z1);
            issue_ring(z + 1 < z1 ? z + 1 : z1 - 1);
            update_plane(L + b * ULP, pm, pc, pp);
            // vmcnt(0) here: the loads above and the previous plane's stores
            // are all that is outstanding (the outputs are conditional, so the
            // compiler would otherwise place the wait after this plane's
            // stores, where it drains them too)
            __builtin_amdgcn_s_waitcnt(VMCNT0);
            store_plane(z);
            b ^= 1;
#pragma unroll
            for (int r = 0; r < URYT; ++r) {
                pm[r] = pc[r];
                pc[r] = pp[r];
                pp[r] = own_val(r);
            }
            stage(L + b * ULP, pc);
            __syncthreads();
        }
    }
}

__global__ void k_pop_moment(int q, int64_t ps, int64_t n, const double *__restrict__ f,
                             double *__restrict__ phi)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = f[i];
    for (int k = 1; k < q; ++k) v += f[k * ps + i];
    phi[i] = v;
}

__global__ void k_pop_equilibrium(int q, int64_t ps, int64_t n, double w0, double w1,
                                  const double *__restrict__ phi, double *__restrict__ f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p = phi[i];
    f[i] = w0 * p;
    for (int k = 1; k < q; ++k) f[k * ps + i] = w1 * p;
}

constexpr int POP_ZCHUNK = 128;  // planes per workgroup in 3D

// mode: 0 one thread per node; 1 tiled, phi summed in the tile (fused);
// 2 split: k_pop_moment writes phi to `phi`, then the tiled update reads it;
// 3 carried: the tiled update reads phi from `phi` and writes phi of the new
// populations to phi_next.
template <int D, int BC, int RV>
hipError_t launch_pop_t(const Shape &s, const PopCoef &c, const double *fin, double *fout, int mode,
                        double *phi, double *phi_next, hipStream_t st)
{
    const int64_t n = s.M0 * s.M1 * s.M2;
    if (mode == 0 || D == 1) {
        hipLaunchKernelGGL((k_pop_direct<D, BC, RV>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           st, s, c, fin, fout);
        return hipGetLastError();
    }
    if constexpr (D >= 2) {
        using T = PopTileDefault;
        const int64_t chunks = (D == 3) ? (s.M0 + POP_ZCHUNK - 1) / POP_ZCHUNK : 1;
        const int utx = (int)((s.M2 + T::UX - 1) / T::UX);
        const int uty = (int)((s.M1 + T::UOY - 1) / T::UOY);
        const int64_t ublk = (int64_t)utx * uty * chunks;
        if (mode == 1) {
            hipLaunchKernelGGL((k_pop_update<T, D, BC, RV, true, false>), dim3((unsigned)ublk), dim3(T::UNT), 0,
                               st, s, c, fin, fout, nullptr, utx, uty, POP_ZCHUNK);
        } else if (mode == 3) {
            hipLaunchKernelGGL((k_pop_update<T, D, BC, RV, false, true>), dim3((unsigned)ublk), dim3(T::UNT), 0,
                               st, s, c, phi, fout, phi_next, utx, uty, POP_ZCHUNK);
        } else {
            hipLaunchKernelGGL(k_pop_moment, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, 2 * D + 1,
                               c.ps, n, fin, phi);
            hipLaunchKernelGGL((k_pop_update<T, D, BC, RV, false, false>), dim3((unsigned)ublk), dim3(T::UNT), 0,
                               st, s, c, phi, fout, nullptr, utx, uty, POP_ZCHUNK);
        }
    }
    return hipGetLastError();
}

template <int D, int BC>
hipError_t launch_pop_nit(const Shape &s, const PopCoef &c, const double *fin, double *fout, int mode,
                          double *phi, double *phi_next, hipStream_t st)
{
    switch (root_variant(c.sc)) {
    case 1: return launch_pop_t<D, BC, 1>(s, c, fin, fout, mode, phi, phi_next, st);
    case 2: return launch_pop_t<D, BC, 2>(s, c, fin, fout, mode, phi, phi_next, st);
    case 3: return launch_pop_t<D, BC, 3>(s, c, fin, fout, mode, phi, phi_next, st);
    case 5: return launch_pop_t<D, BC, 5>(s, c, fin, fout, mode, phi, phi_next, st);
    case 6: return launch_pop_t<D, BC, 6>(s, c, fin, fout, mode, phi, phi_next, st);
    default: return launch_pop_t<D, BC, 0>(s, c, fin, fout, mode, phi, phi_next, st);
    }
}

template <int D>
hipError_t launch_pop_bc(const Shape &s, const PopCoef &c, const double *fin, double *fout, int mode,
                         double *phi, double *phi_next, hipStream_t st)
{
    switch (s.bc) {
    case BC_HN: return launch_pop_nit<D, BC_HN>(s, c, fin, fout, mode, phi, phi_next, st);
    case BC_HD: return launch_pop_nit<D, BC_HD>(s, c, fin, fout, mode, phi, phi_next, st);
    case BC_P: return launch_pop_nit<D, BC_P>(s, c, fin, fout, mode, phi, phi_next, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pop_step(const Shape &s, const PopCoef &c, const double *fin, double *fout, int mode,
                           double *phi, double *phi_next, hipStream_t st)
{
    switch (s.d) {
    case 1: return launch_pop_bc<1>(s, c, fin, fout, mode, phi, phi_next, st);
    case 2: return launch_pop_bc<2>(s, c, fin, fout, mode, phi, phi_next, st);
    case 3: return launch_pop_bc<3>(s, c, fin, fout, mode, phi, phi_next, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace ace

using namespace ace;

struct ace_pop {
    Problem p;
    Shape shape;
    PopCoef c;
    double omega1 = 0.0, s = 0.0;
    int q = 0;
    double *f[2] = {nullptr, nullptr};
    double *phi = nullptr;  // zeroth moment / staging of phi0
    int cur = 0;
    // carried form: phi of f[cur] in carry[ccur] while carry_ok
    double *carry[2] = {nullptr, nullptr};
    int ccur = 0;
    int carry_ok = 0;
    int kernel = ACE_POP_AUTO;
    hipStream_t stream = nullptr;
    int64_t steps = 0;
};

namespace {

// launch mode of launch_pop_step for the handle's kernel choice
int pop_mode(const ace_pop *P)
{
    if (P->p.d == 1 || P->kernel == ACE_POP_DIRECT) return 0;
    if (P->kernel == ACE_POP_SPLIT) return 2;
    if (P->kernel == ACE_POP_FUSED) return 1;
    return 3;  // carried (also the automatic choice for d >= 2)
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

int ace_pop_create(int d, const int64_t *N, const double *L, const double *R, double eps, double dt,
                   int bc, double omega1, ace_pop **out)
{
    if (!out) return ACE_E_ARG;
    *out = nullptr;
    Problem p;
    const int rc = derive(d, N, L, R, eps, dt, bc, p);
    if (rc < 0) return rc;
    if (omega1 == 0.0) omega1 = (d == 1) ? 1.0 / 3.0 : (d == 2 ? 1.0 / 5.0 : 1.0 / 6.0);
    if (!(omega1 > 0.0) || omega1 > 1.0 / (2.0 * d) * (1.0 + 1e-15)) return ACE_E_ARG;
    ace_pop *P = new (std::nothrow) ace_pop();
    if (!P) return ACE_E_NOMEM;
    P->p = p;
    P->shape = shape_of(p);
    P->omega1 = omega1;
    P->s = omega1 / p.kappa;  // kappa = omega_1 / s
    P->q = 2 * d + 1;
    P->c.sc = coef_of(p);
    P->c.w0 = 1.0 - 2.0 * d * omega1;
    P->c.w1 = omega1;
    P->c.A = omega1 * (1.0 - P->s) / P->s;
    // arrays 256-byte aligned and staggered by 1280 bytes, so the 2d+1
    // streams of a wavefront do not start on the same HBM channel
    P->c.ps = (p.total + 31) / 32 * 32 + 160;
    const size_t bytes = sizeof(double) * (size_t)P->q * (size_t)P->c.ps;
    hipError_t e = hipMalloc((void **)&P->f[0], bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&P->f[1], bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&P->phi, sizeof(double) * (size_t)p.total);
    for (int b = 0; b < 2 && e == hipSuccess && d >= 2; ++b)
        e = hipMalloc((void **)&P->carry[b], sizeof(double) * (size_t)p.total);
    if (e != hipSuccess) {
        ace_pop_destroy(P);
        return hip_status(e);
    }
    *out = P;
    return rc;
}

int ace_pop_destroy(ace_pop *P)
{
    if (!P) return ACE_E_ARG;
    if (P->f[0]) (void)hipFree(P->f[0]);
    if (P->f[1]) (void)hipFree(P->f[1]);
    if (P->phi) (void)hipFree(P->phi);
    for (double *b : P->carry)
        if (b) (void)hipFree(b);
    delete P;
    return ACE_OK;
}

int ace_pop_info(const ace_pop *P, int64_t M[3], int64_t *total, int *q, double *omega1, double *s,
                 int64_t *device_bytes)
{
    if (!P) return ACE_E_ARG;
    if (M)
        for (int j = 0; j < 3; ++j) M[j] = P->p.M[j];
    if (total) *total = P->p.total;
    if (q) *q = P->q;
    if (omega1) *omega1 = P->omega1;
    if (s) *s = P->s;
    if (device_bytes)
        *device_bytes = (int64_t)sizeof(double) *
                        (2 * (int64_t)P->q * P->c.ps + P->p.total * (P->carry[0] ? 3 : 1));
    return ACE_OK;
}

int ace_pop_set_stream(ace_pop *P, void *st)
{
    if (!P) return ACE_E_ARG;
    P->stream = (hipStream_t)st;
    return ACE_OK;
}

int ace_pop_set_kernel(ace_pop *P, int kernel)
{
    if (!P || kernel < ACE_POP_AUTO || kernel > ACE_POP_CARRY) return ACE_E_ARG;
    P->kernel = kernel;
    return ACE_OK;
}

int ace_pop_set_phi0(ace_pop *P, const double *phi0, int where)
{
    if (!P || !phi0 || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    const int64_t n = P->p.total;
    const size_t bytes = sizeof(double) * (size_t)n;
    if (where == ACE_HOST) {
        for (int64_t i = 0; i < n; ++i)
            if (!isfinite(phi0[i])) return ACE_E_NONFINITE;
        hipError_t e = hipMemcpyAsync(P->phi, phi0, bytes, hipMemcpyHostToDevice, P->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
        if (e != hipSuccess) return hip_status(e);
    } else {
        hipError_t e = hipMemcpyAsync(P->phi, phi0, bytes, hipMemcpyDeviceToDevice, P->stream);
        if (e != hipSuccess) return hip_status(e);
    }
    hipLaunchKernelGGL(k_pop_equilibrium, dim3(blocks_for(n)), dim3(256), 0, P->stream, P->q, P->c.ps, n,
                       P->c.w0, P->c.w1, P->phi, P->f[P->cur]);
    P->steps = 0;
    P->carry_ok = 0;
    return hip_status(hipGetLastError());
}

int ace_pop_set_populations(ace_pop *P, const double *f, int where)
{
    if (!P || !f || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    const size_t row = sizeof(double) * (size_t)P->p.total;
    hipError_t e = hipMemcpy2DAsync(P->f[P->cur], sizeof(double) * (size_t)P->c.ps, f, row, row,
                                    (size_t)P->q,
                                    where == ACE_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                    P->stream);
    if (e == hipSuccess && where == ACE_HOST) e = hipStreamSynchronize(P->stream);
    P->steps = 0;
    P->carry_ok = 0;
    return hip_status(e);
}

int ace_pop_get_populations(const ace_pop *P, double *f, int where)
{
    if (!P || !f || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    const size_t row = sizeof(double) * (size_t)P->p.total;
    hipError_t e = hipMemcpy2DAsync(f, row, P->f[P->cur], sizeof(double) * (size_t)P->c.ps, row,
                                    (size_t)P->q,
                                    where == ACE_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                    P->stream);
    if (e == hipSuccess && where == ACE_HOST) e = hipStreamSynchronize(P->stream);
    return hip_status(e);
}

int ace_pop_step(ace_pop *P, int64_t nsteps)
{
    if (!P || nsteps < 0) return ACE_E_ARG;
    const int mode = pop_mode(P);
    if (nsteps > 0 && mode == 3 && !P->carry_ok) {  // phi of the current populations, once
        const int64_t n = P->p.total;
        hipLaunchKernelGGL(k_pop_moment, dim3(blocks_for(n)), dim3(256), 0, P->stream, P->q, P->c.ps, n,
                           P->f[P->cur], P->carry[P->ccur]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_status(e);
        P->carry_ok = 1;
    }
    for (int64_t t = 0; t < nsteps; ++t) {
        hipError_t e = launch_pop_step(P->shape, P->c, P->f[P->cur], P->f[P->cur ^ 1], mode,
                                       mode == 3 ? P->carry[P->ccur] : P->phi,
                                       mode == 3 ? P->carry[P->ccur ^ 1] : nullptr, P->stream);
        if (e != hipSuccess) return hip_status(e);
        P->cur ^= 1;
        if (mode == 3) P->ccur ^= 1;
        ++P->steps;
    }
    if (nsteps > 0 && mode != 3) P->carry_ok = 0;
    return ACE_OK;
}

int ace_pop_get_phi(ace_pop *P, double *phi, int where)
{
    if (!P || !phi || (where != ACE_HOST && where != ACE_DEVICE)) return ACE_E_ARG;
    const int64_t n = P->p.total;
    double *dst = (where == ACE_DEVICE) ? phi : P->phi;
    hipLaunchKernelGGL(k_pop_moment, dim3(blocks_for(n)), dim3(256), 0, P->stream, P->q, P->c.ps, n,
                       P->f[P->cur], dst);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && where == ACE_HOST) {
        e = hipMemcpyAsync(phi, P->phi, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, P->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    }
    return hip_status(e);
}

int64_t ace_pop_step_count(const ace_pop *P) { return P ? P->steps : -1; }

}  // extern "C"
