// 3D step kernel: each workgroup owns a TY x TX tile of the two fastest axes
// (i1, i2) and a chunk of planes along the slowest axis i0, and marches
// through the chunk one plane at a time.  The current plane of the tile plus
// a one-node ring sits in LDS (double-buffered, one barrier per plane); the
// i0 neighbours come from a per-thread register queue that is prefetched two
// planes ahead, so each interior value is read from HBM once per step.
//
// Boundary values are folded into the data movement: every ring slot and every
// plane outside the domain holds the value the BC assigns to that neighbour
// (Neumann: the clamped node, i.e. the node itself; Dirichlet: 0; periodic:
// the wrapped node), so the update itself has no boundary branches.
#include "ace_device.h"

namespace ace {

namespace {

constexpr int TX = 64;        // tile width along i2 (one wavefront)
constexpr int TROWS = 4;      // thread rows per workgroup
constexpr int RY = 4;         // tile rows per thread row
constexpr int TY = TROWS * RY;
constexpr int NT = TX * TROWS;  // 256 threads
constexpr int ZCHUNK = 64;    // planes per workgroup
constexpr int LW = TX + 2;    // LDS row width

// Coordinate of the neighbour at c under BC, or -1 when the neighbour is the
// Dirichlet zero.  Coordinates more than one past either end only occur for
// slots no in-domain node reads; they are mapped to any in-range node.
template <int BC>
__device__ __forceinline__ int64_t map_coord(int64_t c, int64_t n)
{
    if (c >= 0 && c < n) return c;
    if (BC == BC_HN) return c < 0 ? 0 : n - 1;
    if (BC == BC_HD) return -1;
    if (c < 0) return n - 1;
    return c - n < n ? c - n : 0;
}

// Offset of (y, x) inside a plane under the BC, or -1 for the Dirichlet zero.
template <int BC>
__device__ __forceinline__ int64_t plane_offset(const Shape &s, int64_t y, int64_t x)
{
    const int64_t my = map_coord<BC>(y, s.M1);
    const int64_t mx = map_coord<BC>(x, s.M2);
    if (my < 0 || mx < 0) return -1;
    return my * s.M2 + mx;
}

// Start of plane z under the BC, or -1 for a Dirichlet zero plane.
template <int BC>
__device__ __forceinline__ int64_t plane_base(const Shape &s, int64_t z)
{
    const int64_t mz = map_coord<BC>(z, s.M0);
    return mz < 0 ? -1 : mz * s.M1 * s.M2;
}

__device__ __forceinline__ double load_at(const double *__restrict__ in, int64_t base, int64_t off)
{
    return (base < 0 || off < 0) ? 0.0 : in[base + off];
}

template <int BC, bool MON>
__global__ __launch_bounds__(NT) void k_march3d(Shape s, StepCoef c, const double *__restrict__ in,
                                                double *__restrict__ out,
                                                double *__restrict__ partials, int tiles_x,
                                                int tiles_y, int nchunks)
{
    __shared__ double lds[2][TY + 2][LW];
    __shared__ double red[3 * (NT / 64)];
    (void)nchunks;

    const int64_t t = xcd_tile(blockIdx.x, gridDim.x);  // XCD-aware numbering
    const int64_t ntile = (int64_t)tiles_x * tiles_y;
    const int tile_xy = (int)(t % ntile);
    const int chunk = (int)(t / ntile);
    const int tile_x = tile_xy % tiles_x;
    const int tile_y = tile_xy / tiles_x;

    const int tx = threadIdx.x & (TX - 1);
    const int tr = threadIdx.x / TX;
    const int64_t x = (int64_t)tile_x * TX + tx;
    const int64_t ybase = (int64_t)tile_y * TY + tr * RY;
    const int64_t z0 = (int64_t)chunk * ZCHUNK;
    const int64_t z1 = (z0 + ZCHUNK < s.M0) ? z0 + ZCHUNK : s.M0;
    const int64_t PS = s.M1 * s.M2;

    // In-plane offsets of this thread's RY nodes (BC-mapped for slots past
    // the domain) and of its ring slot: threads 0..2TX-1 own the rows above
    // and below the tile, threads 2TX..2TX+2TY-1 the columns left and right.
    int64_t off[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) off[r] = plane_offset<BC>(s, ybase + r, x);
    int ring_ly = -1, ring_lx = -1;
    int64_t roff = -1;
    {
        const int t0 = threadIdx.x;
        int64_t ry = 0, rx = 0;
        if (t0 < 2 * TX) {
            ring_ly = (t0 < TX) ? 0 : TY + 1;
            ring_lx = (t0 & (TX - 1)) + 1;
        } else if (t0 < 2 * TX + 2 * TY) {
            const int u = t0 - 2 * TX;
            ring_lx = (u < TY) ? 0 : TX + 1;
            ring_ly = (u % TY) + 1;
        }
        if (ring_ly >= 0) {
            ry = (int64_t)tile_y * TY + ring_ly - 1;
            rx = (int64_t)tile_x * TX + ring_lx - 1;
            roff = plane_offset<BC>(s, ry, rx);
        }
    }
    const bool has_ring = ring_ly >= 0;

    // register queue: q0 = plane z-1, q1 = z, q2 = z+1, q3 = z+2 (in flight)
    double q0[RY], q1[RY], q2[RY], q3[RY];
    const int64_t bm1 = plane_base<BC>(s, z0 - 1), b0 = plane_base<BC>(s, z0);
    const int64_t b1 = plane_base<BC>(s, z0 + 1);
    const int64_t b2 = (z0 + 2 <= z1) ? plane_base<BC>(s, z0 + 2) : -1;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        q0[r] = load_at(in, bm1, off[r]);
        q1[r] = load_at(in, b0, off[r]);
        q2[r] = load_at(in, b1, off[r]);
        q3[r] = load_at(in, b2, off[r]);
    }
    double r2 = 0.0;  // ring value of plane z+1
    if (has_ring) {
        lds[0][ring_ly][ring_lx] = load_at(in, b0, roff);
        r2 = load_at(in, b1, roff);
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) lds[0][tr * RY + r + 1][tx + 1] = q1[r];
    __syncthreads();

    MonAcc m;
    mon_zero(m);
    const bool xin = x < s.M2;
    int buf = 0;
    for (int64_t z = z0; z < z1; ++z) {
        // --- update plane z: i1/i2 neighbours from LDS, i0 from registers ---
        double *const orow = out + z * PS;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int ly = tr * RY + r + 1;
            const double p = q1[r];
            const double xm = lds[buf][ly][tx];
            const double xp = lds[buf][ly][tx + 2];
            const double ym = (r > 0) ? q1[r > 0 ? r - 1 : 0] : lds[buf][ly - 1][tx + 1];
            const double yp = (r < RY - 1) ? q1[r < RY - 1 ? r + 1 : 0] : lds[buf][ly + 1][tx + 1];
            const double nsum = ((q0[r] + q2[r]) + (ym + yp)) + (xm + xp);
            const int64_t y = ybase + r;
            if (xin && y < s.M1) {
                orow[y * s.M2 + x] = update<3>(p, nsum, c);
                if (MON) {
                    const double dz = q2[r] - p, dy = yp - p, dx = xp - p;
                    double g = fma(dz, dz, fma(dy, dy, dx * dx));
                    if (BC == BC_HD) {
                        if (z == 0) g = fma(p, p, g);
                        if (y == 0) g = fma(p, p, g);
                        if (x == 0) g = fma(p, p, g);
                    }
                    m.bulk += bulk_term(p);
                    m.grad += g;
                    m.mx = nan_max(m.mx, fabs(p));
                }
            }
        }
        if (z + 1 >= z1) break;
        // --- advance the queue and stage plane z+1 in the other buffer ---
        const int64_t b3 = (z + 3 <= z1) ? plane_base<BC>(s, z + 3) : -1;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q0[r] = q1[r];
            q1[r] = q2[r];
            q2[r] = q3[r];
            q3[r] = load_at(in, b3, off[r]);
        }
        const double rn = r2;
        if (has_ring && z + 2 < z1) r2 = load_at(in, plane_base<BC>(s, z + 2), roff);
        buf ^= 1;
#pragma unroll
        for (int r = 0; r < RY; ++r) lds[buf][tr * RY + r + 1][tx + 1] = q1[r];
        if (has_ring) lds[buf][ring_ly][ring_lx] = rn;
        __syncthreads();
    }
    if (MON) block_reduce_store(m, red, partials + 3 * t);
}

}  // namespace

bool march_supported(const Shape &s)
{
    return s.d == 3 && s.M0 >= 1 && s.M1 >= 1 && s.M2 >= 1;
}

int64_t march_partials_needed(const Shape &s)
{
    return ((s.M2 + TX - 1) / TX) * ((s.M1 + TY - 1) / TY) * ((s.M0 + ZCHUNK - 1) / ZCHUNK);
}

hipError_t launch_step_march(const Shape &s, const StepCoef &c, const double *in, double *out,
                             double *partials, int64_t *nparts, hipStream_t st)
{
    if (!march_supported(s)) return hipErrorInvalidValue;
    const int tiles_x = (int)((s.M2 + TX - 1) / TX);
    const int tiles_y = (int)((s.M1 + TY - 1) / TY);
    const int nchunks = (int)((s.M0 + ZCHUNK - 1) / ZCHUNK);
    const int64_t nblk = (int64_t)tiles_x * tiles_y * nchunks;
    if (nparts) *nparts = nblk;
#define ACE_MARCH(BB)                                                                          \
    if (s.bc == BB) {                                                                          \
        if (partials)                                                                          \
            hipLaunchKernelGGL((k_march3d<BB, true>), dim3((unsigned)nblk), dim3(NT), 0, st, s, \
                               c, in, out, partials, tiles_x, tiles_y, nchunks);               \
        else                                                                                   \
            hipLaunchKernelGGL((k_march3d<BB, false>), dim3((unsigned)nblk), dim3(NT), 0, st,   \
                               s, c, in, out, partials, tiles_x, tiles_y, nchunks);            \
        return hipGetLastError();                                                              \
    }
    ACE_MARCH(BC_HN) ACE_MARCH(BC_HD) ACE_MARCH(BC_P)
#undef ACE_MARCH
    return hipErrorInvalidValue;
}

}  // namespace ace
