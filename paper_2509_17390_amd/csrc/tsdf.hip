// tsdf.hip -- denoising, flood-fill sign, narrow-band TSDF and marching cubes
// on gfx950 (FGGS-LiDAR Sec. IV-B).
//
//   V'    = G * V (binomial kernel of n steps: integer weights C(2n, n+k),
//           the discrete Gaussian of variance n / 2), separable, exact in
//           64-bit integers; V~ = [V' >= tau], decided on the exact sum
//   O     = free voxels 6-connected to a free frame around the grid:
//           rounds of line sweeps along x, y and z (one thread per line,
//           spreading along whole free runs) until a round changes nothing
//   S_0   = voxels with a 6-neighbour of the other V~ value (frame = free)
//   p     = shell index of a 6-neighbour expansion from S_0, up to ceil(r / h)
//           shells: for at most 4, S_0, the shells and phi in one pass over
//           LDS tiles; else one launch each
//   phi   = clip(s p h, -r, r), s = +1 on O, -1 elsewhere
//   mesh  = marching cubes of phi at iso on the voxel-centre lattice:
//           per point, count crossed lattice edges (one vertex each) and the
//           triangles of the cell it anchors; tile scans give every vertex
//           and triangle its slot; a second pass writes them.  The case
//           table is built on the host from a walk over the cube's faces.
#include "mesh_internal.h"

#include <math.h>

#include <mutex>

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 4;                  // per thread in the block scan
constexpr int kScanTile = kBlock * kScanItems;

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// (x, y, z) of voxel i.  Below 2^32 voxels the divisions by nx and ny are
// multiplications (64-bit integer division is a long emulated sequence,
// and these kernels run it for every voxel).
__device__ __forceinline__ uint32_t div_by(uint32_t n, uint64_t c)
{
    return c ? (uint32_t)__umul64hi(c, (uint64_t)n) : n;
}

__device__ __forceinline__ void coords(int64_t i, const TsdfGrid &g, int &x, int &y, int &z)
{
    if (g.n <= (int64_t)0xffffffffLL) {
        const uint32_t u = (uint32_t)i;
        const uint32_t r = div_by(u, g.cx);
        x = (int)(u - r * (uint32_t)g.nx);
        const uint32_t zz = div_by(r, g.cy);
        y = (int)(r - zz * (uint32_t)g.ny);
        z = (int)zz;
        return;
    }
    x = (int)(i % g.nx);
    const int64_t r = i / g.nx;
    y = (int)(r % g.ny);
    z = (int)(r / g.ny);
}

// ---- smoothing and re-threshold ------------------------------------------
__global__ __launch_bounds__(kBlock) void k_smooth_x(const uint8_t *__restrict__ v,
                                                     uint32_t *__restrict__ out, TsdfGrid g,
                                                     Binomial w)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int x, y, z;
    coords(i, g, x, y, z);
    uint32_t s = 0;
    for (int k = -w.n; k <= w.n; ++k) {
        const int xx = x + k;
        if (xx >= 0 && xx < g.nx && v[i + k]) s += w.w[k + w.n];
    }
    out[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_smooth_y(const uint32_t *__restrict__ a,
                                                     uint64_t *__restrict__ out, TsdfGrid g,
                                                     Binomial w)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int x, y, z;
    coords(i, g, x, y, z);
    uint64_t s = 0;
    for (int k = -w.n; k <= w.n; ++k) {
        const int yy = y + k;
        if (yy >= 0 && yy < g.ny) s += (uint64_t)w.w[k + w.n] * a[i + (int64_t)k * g.nx];
    }
    out[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_smooth_z(const uint64_t *__restrict__ b,
                                                     uint8_t *__restrict__ vt, TsdfGrid g,
                                                     Binomial w, uint64_t thr)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const int64_t sxy = (int64_t)g.nx * g.ny;
    int x, y, z;
    coords(i, g, x, y, z);
    uint64_t s = 0;
    for (int k = -w.n; k <= w.n; ++k) {
        const int zz = z + k;
        if (zz >= 0 && zz < g.nz) s += (uint64_t)w.w[k + w.n] * b[i + (int64_t)k * sxy];
    }
    vt[i] = s >= thr ? 1 : 0;
}

// The same z pass keeping the integer sums (for the quantile re-threshold),
// and the threshold of such sums against a value held on the device.
__global__ __launch_bounds__(kBlock) void k_smooth_z_sum(const uint64_t *__restrict__ b,
                                                         uint64_t *__restrict__ out, TsdfGrid g,
                                                         Binomial w)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const int64_t sxy = (int64_t)g.nx * g.ny;
    int x, y, z;
    coords(i, g, x, y, z);
    uint64_t s = 0;
    for (int k = -w.n; k <= w.n; ++k) {
        const int zz = z + k;
        if (zz >= 0 && zz < g.nz) s += (uint64_t)w.w[k + w.n] * b[i + (int64_t)k * sxy];
    }
    out[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_threshold_sums(const uint64_t *__restrict__ sums,
                                                           const uint64_t *__restrict__ thr,
                                                           uint8_t *__restrict__ vt, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) vt[i] = sums[i] >= *thr ? 1 : 0;
}

// Fast path for kernels of at most kFastSmooth steps (sums fit u8 after x,
// u16 after y, u32 after z): four voxels per thread, word loads, narrow
// intermediates.  One byte- or word-wide load per lane and tap capped the
// one-voxel passes at the rate the memory pipeline issues instructions.
// The intermediates carry readable padding of three taps plus two words on
// both sides, so no load leaves the buffer; taps outside the grid are
// excluded by coordinates, never by the values read.
constexpr int kFastSmooth = 3;

__device__ __forceinline__ uint32_t word_at(const uint8_t *__restrict__ p, int64_t idx)
{
    const int64_t a = idx & ~(int64_t)3;
    const uint32_t lo = *reinterpret_cast<const uint32_t *>(p + a);
    const int sh = (int)(idx & 3);
    if (sh == 0) return lo;
    const uint32_t hi = *reinterpret_cast<const uint32_t *>(p + a + 4);
    return __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)sh);
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int j) { return (w >> (8 * j)) & 0xffu; }

__device__ __forceinline__ uint32_t word_guarded(const uint8_t *__restrict__ p, int64_t idx,
                                                 int64_t n)
{
    // bytes idx .. idx + 3 of p[0, n) (0 outside it); idx is a multiple of 4
    if (idx >= 0 && idx + 4 <= n) return *reinterpret_cast<const uint32_t *>(p + idx);
    uint32_t w = 0;
    for (int j = 0; j < 4; ++j) {
        const int64_t q = idx + j;
        if (q >= 0 && q < n) w |= (uint32_t)p[q] << (8 * j);
    }
    return w;
}

// the 8 bytes at byte offset off (even) of a padded buffer
__device__ __forceinline__ void bytes8_at(const uint8_t *__restrict__ p, int64_t off,
                                          uint32_t &lo, uint32_t &hi)
{
    const int64_t a = off & ~(int64_t)3;
    const uint32_t d0 = *reinterpret_cast<const uint32_t *>(p + a);
    const uint32_t d1 = *reinterpret_cast<const uint32_t *>(p + a + 4);
    if ((off & 3) == 0) {
        lo = d0;
        hi = d1;
        return;
    }
    const uint32_t d2 = *reinterpret_cast<const uint32_t *>(p + a + 8);
    lo = __builtin_amdgcn_alignbyte(d1, d0, 2u);
    hi = __builtin_amdgcn_alignbyte(d2, d1, 2u);
}

__device__ __forceinline__ void step_voxel(const TsdfGrid &g, int &x, int &y, int &z)
{
    if (++x == g.nx) {
        x = 0;
        if (++y == g.ny) {
            y = 0;
            ++z;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_smooth_x4(const uint8_t *__restrict__ v,
                                                      uint8_t *__restrict__ a8, TsdfGrid g,
                                                      Binomial w)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i0 >= g.n) return;
    // bytes i0 - 4 .. i0 + 7 cover the taps of the four voxels
    const uint32_t w0 = word_guarded(v, i0 - 4, g.n), w1 = word_guarded(v, i0, g.n),
                   w2 = word_guarded(v, i0 + 4, g.n);
    int x, y, z;
    coords(i0, g, x, y, z);
    uint32_t out = 0;
    for (int j = 0; j < 4; ++j) {
        uint32_t sum = 0;
        for (int k = -w.n; k <= w.n; ++k) {
            const int xx = x + k;
            if (xx < 0 || xx >= g.nx) continue;
            const int pos = 4 + j + k;                  // 1 .. 10
            const uint32_t wd = pos < 4 ? w0 : (pos < 8 ? w1 : w2);
            if ((wd >> (8 * (pos & 3))) & 0xffu) sum += w.w[k + w.n];
        }
        out |= sum << (8 * j);
        step_voxel(g, x, y, z);
    }
    *reinterpret_cast<uint32_t *>(a8 + i0) = out;
}

__global__ __launch_bounds__(kBlock) void k_smooth_y4(const uint8_t *__restrict__ a8,
                                                      uint16_t *__restrict__ b16, TsdfGrid g,
                                                      Binomial w)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i0 >= g.n) return;
    int x, y, z;
    coords(i0, g, x, y, z);
    int yj[4];
    for (int j = 0; j < 4; ++j) {
        yj[j] = y;
        step_voxel(g, x, y, z);
    }
    uint32_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int k = -w.n; k <= w.n; ++k) {
        const uint32_t wd = word_at(a8, i0 + (int64_t)k * g.nx);
        const uint32_t c = w.w[k + w.n];
        if ((unsigned)(yj[0] + k) < (unsigned)g.ny) s0 += c * (wd & 0xffu);
        if ((unsigned)(yj[1] + k) < (unsigned)g.ny) s1 += c * ((wd >> 8) & 0xffu);
        if ((unsigned)(yj[2] + k) < (unsigned)g.ny) s2 += c * ((wd >> 16) & 0xffu);
        if ((unsigned)(yj[3] + k) < (unsigned)g.ny) s3 += c * (wd >> 24);
    }
    *reinterpret_cast<uint2 *>(b16 + i0) = make_uint2(s0 | (s1 << 16), s2 | (s3 << 16));
}

__global__ __launch_bounds__(kBlock) void k_smooth_z4(const uint8_t *__restrict__ b8,
                                                      uint8_t *__restrict__ vt, TsdfGrid g,
                                                      Binomial w, uint64_t thr)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i0 >= g.n) return;
    const int64_t sxy = (int64_t)g.nx * g.ny;
    int x, y, z;
    coords(i0, g, x, y, z);
    int zj[4];
    for (int j = 0; j < 4; ++j) {
        zj[j] = z;
        step_voxel(g, x, y, z);
    }
    uint32_t s[4] = {0, 0, 0, 0};
    for (int k = -w.n; k <= w.n; ++k) {
        uint32_t lo, hi;
        bytes8_at(b8, 2 * (i0 + (int64_t)k * sxy), lo, hi);
        const uint32_t c = w.w[k + w.n];
        const uint32_t v4[4] = {lo & 0xffffu, lo >> 16, hi & 0xffffu, hi >> 16};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((unsigned)(zj[j] + k) < (unsigned)g.nz) s[j] += c * v4[j];
    }
    uint32_t out = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) out |= ((uint64_t)s[j] >= thr ? 1u : 0u) << (8 * j);
    if (i0 + 4 <= g.n) {
        *reinterpret_cast<uint32_t *>(vt + i0) = out;
    } else {
        for (int j = 0; i0 + j < g.n; ++j) vt[i0 + j] = (uint8_t)((out >> (8 * j)) & 0xffu);
    }
}

// Smoothing, threshold and packing in one pass over 64 x 8 x 8 tiles, for
// kernels of at most 3 steps: a block loads the surface bytes over its tile
// with a halo of n voxels (0 outside the grid, which is what the per-grid
// passes' skipped taps add), forms the x sums (u8), the x-y sums (u16) and
// the full sums in LDS in the same integer arithmetic, writes V~ and, one
// wave per row, the row's free word (the tile's 64 columns are one word)
// with a clear outside word.
constexpr int kSmTX = 64, kSmTY = 8, kSmTZ = 8;
constexpr int kLoadBatch = 8;

template <int N>
__global__ __launch_bounds__(kBlock) void k_smooth_pack_tile(const uint8_t *__restrict__ surf,
                                                             uint8_t *__restrict__ vt, TsdfGrid g,
                                                             Binomial w, uint64_t thr, int W,
                                                             uint64_t *__restrict__ F,
                                                             uint64_t *__restrict__ O)
{
    static_assert(N >= 1 && N <= 3, "u8 x sums: at most 2^(2N) <= 64");
    constexpr int SX = kSmTX + 2 * N, SY = kSmTY + 2 * N, SZ = kSmTZ + 2 * N;
    constexpr int NS = SX * SY * SZ;                      // surface bytes
    constexpr int NA = kSmTX * SY * SZ;                   // x sums, u8
    constexpr int NB = kSmTX * kSmTY * SZ;                // x-y sums, u16
    constexpr int R1 = NS > 2 * NB ? NS : 2 * NB;
    // the surface bytes are dead once the x sums exist: the x-y sums reuse
    // their space
    __shared__ __align__(16) uint8_t r1[R1];
    __shared__ uint8_t A[NA];
    uint8_t *S = r1;
    uint16_t *B = reinterpret_cast<uint16_t *>(r1);
    const int bx = (int)blockIdx.x * kSmTX, by = (int)blockIdx.y * kSmTY;
    const int bz = (int)blockIdx.z * kSmTZ;
    // kLoadBatch loads per thread in flight at once: a voxel outside the
    // grid reads voxel 0 (always there) and counts as 0, so no branch
    // separates a load from the next
    for (int q0 = threadIdx.x; q0 < NS; q0 += kLoadBatch * kBlock) {
        uint8_t v[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
            const int q = q0 + k * kBlock;
            const int lx = q % SX, t = q / SX, ly = t % SY, lz = t / SY;
            const int gx = bx - N + lx, gy = by - N + ly, gz = bz - N + lz;
            const bool ok = q < NS && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 &&
                            gz < g.nz;
            v[k] = surf[ok ? ((int64_t)gz * g.ny + gy) * g.nx + gx : 0];
            v[k] = ok && v[k] != 0 ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k)
            if (q0 + k * kBlock < NS) S[q0 + k * kBlock] = v[k];
    }
    __syncthreads();
    const int lx = (int)threadIdx.x % kSmTX, r0 = (int)threadIdx.x / kSmTX;
    constexpr int RPI = kBlock / kSmTX;                   // rows per round
    for (int r = r0; r < SY * SZ; r += RPI) {             // row (ly, lz) of the halo'd tile
        const uint8_t *src = S + r * SX + lx;
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k <= 2 * N; ++k) sum += w.w[k] * src[k];
        A[r * kSmTX + lx] = (uint8_t)sum;
    }
    __syncthreads();
    for (int r = r0; r < kSmTY * SZ; r += RPI) {          // ly in [0, TY), lz in [0, SZ)
        const int ly = r % kSmTY, lz = r / kSmTY;
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k <= 2 * N; ++k) sum += w.w[k] * A[(lz * SY + ly + k) * kSmTX + lx];
        B[r * kSmTX + lx] = (uint16_t)sum;
    }
    __syncthreads();
    const int gx = bx + lx;
    for (int r = r0; r < kSmTY * kSmTZ; r += RPI) {       // one wave per output row
        const int ly = r % kSmTY, lz = r / kSmTY;
        const int gy = by + ly, gz = bz + lz;
        if (gy >= g.ny || gz >= g.nz) continue;           // the whole wave
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k <= 2 * N; ++k)
            sum += w.w[k] * B[((lz + k) * kSmTY + ly) * kSmTX + lx];
        const bool in = gx < g.nx;
        const bool v = in && (uint64_t)sum >= thr;
        const int64_t row = (int64_t)gz * g.ny + gy;
        if (in) vt[row * g.nx + gx] = v ? 1 : 0;
        const uint64_t f = __ballot(in && !v);
        if (lx == 0) {
            F[row * W + blockIdx.x] = f;
            O[row * W + blockIdx.x] = 0;
        }
    }
}

// ---- outside labelling -----------------------------------------------------
// Bit-packed along x: word (z, y, wx) holds voxels x = 64 wx .. 64 wx + 63
// of row (y, z); F = free (V~ = 0), O = known to be outside; bits beyond
// nx are never free.  A sweep along an axis makes every run of free voxels
// on a line that holds an outside voxel or touches the frame (beyond both
// ends of the line) outside; sweeps along x, y and z repeat until a round
// changes nothing, which is the 6-connected component joined to the frame
// (a path to the frame is a chain of axis-parallel runs).  O only grows.
//
// x: one thread per row, an occluded fill per word with a carry bit.
// y and z: 64 lines per thread (one word column), where one row step is
// R = F & (R | O).  Lines are cut into kSegRows-row segments for
// parallelism: (1) per segment, the reach out of its end and out of its
// start from its own seeds, and the lines it is free on throughout; (2) per
// column, the carries into each segment from the frame and the segments
// before and after it; (3) per segment, the walk forward from its left
// carry and backward from its right carry.
constexpr int kSegRows = 16;

__device__ __forceinline__ uint64_t fill_up(uint64_t gen, uint64_t pro)
{
    gen |= pro & (gen << 1);
    pro &= pro << 1;
    gen |= pro & (gen << 2);
    pro &= pro << 2;
    gen |= pro & (gen << 4);
    pro &= pro << 4;
    gen |= pro & (gen << 8);
    pro &= pro << 8;
    gen |= pro & (gen << 16);
    pro &= pro << 16;
    gen |= pro & (gen << 32);
    return gen;
}

__device__ __forceinline__ uint64_t fill_down(uint64_t gen, uint64_t pro)
{
    gen |= pro & (gen >> 1);
    pro &= pro >> 1;
    gen |= pro & (gen >> 2);
    pro &= pro >> 2;
    gen |= pro & (gen >> 4);
    pro &= pro >> 4;
    gen |= pro & (gen >> 8);
    pro &= pro >> 8;
    gen |= pro & (gen >> 16);
    pro &= pro >> 16;
    gen |= pro & (gen >> 32);
    return gen;
}

// one wave per word: lane b reads voxel 64 wx + b (coalesced), a ballot
// packs the word
__global__ __launch_bounds__(kBlock) void k_pack_free(const uint8_t *__restrict__ vt, TsdfGrid g,
                                                      int W, uint64_t *__restrict__ F,
                                                      uint64_t *__restrict__ O)
{
    const int64_t w = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)W * g.ny * g.nz;
    if (w >= nw) return;                                  // whole waves
    const int lane = (int)(threadIdx.x & 63);
    const int64_t row = w / W;
    const int wx = (int)(w - row * W);
    const int x = wx * 64 + lane;
    const bool free_ = x < g.nx && vt[row * g.nx + x] == 0;
    const uint64_t f = __ballot(free_);
    if (lane == 0) {
        F[w] = f;
        O[w] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_sweep_x(const uint64_t *__restrict__ F,
                                                    uint64_t *__restrict__ O, TsdfGrid g, int W,
                                                    int32_t *__restrict__ changed,
                                                    const int32_t *__restrict__ skip)
{
    // a round enqueued after the labelling settled does nothing
    if (skip && *skip == 0) return;

    const int64_t row = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (row >= (int64_t)g.ny * g.nz) return;
    const uint64_t *f = F + row * W;
    uint64_t *o = O + row * W;
    const int top = (g.nx - 1) & 63;                      // last voxel's bit in the last word
    bool any = false;
    uint64_t carry = 1;                                   // the frame before x = 0
    for (int wx = 0; wx < W; ++wx) {
        const uint64_t fw = f[wx], ow = o[wx];
        const uint64_t gen = fill_up(ow | (fw & carry), fw);
        if (gen != ow) {
            o[wx] = gen;
            any = true;
        }
        carry = gen >> 63;
    }
    carry = 1;                                            // the frame after x = nx - 1
    for (int wx = W - 1; wx >= 0; --wx) {
        const uint64_t fw = f[wx], ow = o[wx];
        const uint64_t seed = carry ? (fw & (1ull << (wx == W - 1 ? top : 63))) : 0ull;
        const uint64_t gen = fill_down(ow | seed, fw);
        if (gen != ow) {
            o[wx] = gen;
            any = true;
        }
        carry = gen & 1ull;
    }
    if (any && *changed == 0) *changed = 1;
}

// word-column layout of a sweep along y (AXIS 1) or z (AXIS 2): column c,
// row r -> word base + r * stride; rows = ny or nz
struct Cols {
    int64_t ncols, stride;
    int rows, nseg;
};

template <int AXIS>
__device__ __forceinline__ int64_t col_base(int64_t c, const TsdfGrid &g, int W)
{
    const int64_t a = c / W, wx = c - a * W;
    return AXIS == 1 ? a * g.ny * W + wx      // a = z
                     : a * W + wx;            // a = y
}

// (1) per segment: A = reach out of its end, B = reach out of its start
// (from its own outside voxels), T = lines free on every row
template <int AXIS>
__global__ __launch_bounds__(kBlock) void k_seg_summary(const uint64_t *__restrict__ F,
                                                        const uint64_t *__restrict__ O,
                                                        TsdfGrid g, int W, Cols cl,
                                                        uint64_t *__restrict__ A,
                                                        uint64_t *__restrict__ B,
                                                        uint64_t *__restrict__ T,
                                                        const int32_t *__restrict__ skip)
{
    // a round enqueued after the labelling settled does nothing
    if (skip && *skip == 0) return;

    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= cl.ncols * cl.nseg) return;
    const int sg = (int)(t / cl.ncols);
    const int64_t c = t - (int64_t)sg * cl.ncols;
    const int64_t base = col_base<AXIS>(c, g, W);
    const int r0 = sg * kSegRows;
    const int nr = cl.rows - r0 < kSegRows ? cl.rows - r0 : kSegRows;
    uint64_t f[kSegRows], o[kSegRows];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k) {
        f[k] = k < nr ? F[base + (int64_t)(r0 + k) * cl.stride] : 0ull;
        o[k] = k < nr ? O[base + (int64_t)(r0 + k) * cl.stride] : 0ull;
    }
    uint64_t r = 0, tr = ~0ull;
#pragma unroll
    for (int k = 0; k < kSegRows; ++k)
        if (k < nr) {
            r = f[k] & (r | o[k]);
            tr &= f[k];
        }
    uint64_t rb = 0;
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k)
        if (k < nr) rb = f[k] & (rb | o[k]);
    A[t] = r;
    B[t] = rb;
    T[t] = tr;
}

// (2) per column: carries into each segment, C from the start side (the
// frame before row 0), D from the end side (the frame after the last row)
__global__ __launch_bounds__(kBlock) void k_seg_carry(const uint64_t *__restrict__ A,
                                                      const uint64_t *__restrict__ B,
                                                      const uint64_t *__restrict__ T, Cols cl,
                                                      uint64_t *__restrict__ C,
                                                      uint64_t *__restrict__ D,
                                                      const int32_t *__restrict__ skip)
{
    // a round enqueued after the labelling settled does nothing
    if (skip && *skip == 0) return;

    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= cl.ncols) return;
    // 8 segments' summaries are loaded together, then chained in registers
    // (one dependent load per segment left the walk latency-bound)
    constexpr int G = 8;
    uint64_t carry = ~0ull;
    for (int s0 = 0; s0 < cl.nseg; s0 += G) {
        uint64_t a[G], t[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int64_t i = (int64_t)(s0 + k) * cl.ncols + c;
            a[k] = s0 + k < cl.nseg ? A[i] : 0ull;
            t[k] = s0 + k < cl.nseg ? T[i] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (s0 + k < cl.nseg) {
                C[(int64_t)(s0 + k) * cl.ncols + c] = carry;
                carry = a[k] | (t[k] & carry);
            }
    }
    carry = ~0ull;
    for (int s1 = cl.nseg - 1; s1 >= 0; s1 -= G) {
        uint64_t b[G], t[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const int64_t i = (int64_t)(s1 - k) * cl.ncols + c;
            b[k] = s1 - k >= 0 ? B[i] : 0ull;
            t[k] = s1 - k >= 0 ? T[i] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (s1 - k >= 0) {
                D[(int64_t)(s1 - k) * cl.ncols + c] = carry;
                carry = b[k] | (t[k] & carry);
            }
    }
}

// (3) per segment: forward from C, backward from D, new outside bits out
template <int AXIS>
__global__ __launch_bounds__(kBlock) void k_seg_apply(const uint64_t *__restrict__ F,
                                                      uint64_t *__restrict__ O, TsdfGrid g,
                                                      int W, Cols cl,
                                                      const uint64_t *__restrict__ C,
                                                      const uint64_t *__restrict__ D,
                                                      int32_t *__restrict__ changed,
                                                      const int32_t *__restrict__ skip)
{
    // a round enqueued after the labelling settled does nothing
    if (skip && *skip == 0) return;

    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= cl.ncols * cl.nseg) return;
    const int sg = (int)(t / cl.ncols);
    const int64_t c = t - (int64_t)sg * cl.ncols;
    const int64_t base = col_base<AXIS>(c, g, W);
    const int r0 = sg * kSegRows;
    const int nr = cl.rows - r0 < kSegRows ? cl.rows - r0 : kSegRows;
    uint64_t f[kSegRows], o[kSegRows], o0[kSegRows];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k) {
        f[k] = k < nr ? F[base + (int64_t)(r0 + k) * cl.stride] : 0ull;
        o[k] = k < nr ? O[base + (int64_t)(r0 + k) * cl.stride] : 0ull;
        o0[k] = o[k];
    }
    uint64_t r = C[t];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k)
        if (k < nr) {
            r = f[k] & (r | o[k]);
            o[k] = r;
        }
    r = D[t];
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k)
        if (k < nr) {
            r = f[k] & (r | o[k]);
            o[k] = r;
        }
    bool any = false;
#pragma unroll
    for (int k = 0; k < kSegRows; ++k)
        if (k < nr && o[k] != o0[k]) {
            O[base + (int64_t)(r0 + k) * cl.stride] = o[k];
            any = true;
        }
    if (any && *changed == 0) *changed = 1;
}

// (1) to (3) in one kernel, for columns of at most kFusedSegs segments: a
// block takes cj adjacent columns (threads column-fastest, so the words of
// one row are read together; cj * nseg <= kBlock), keeps each segment's
// words in registers, and one thread per column chains the summaries
// through LDS into the carries; the same recurrences as the three kernels,
// without two launches and the summary and carry arrays.
constexpr int kFusedSegs = 32;

template <int AXIS>
__global__ __launch_bounds__(kBlock) void k_seg_fused(const uint64_t *__restrict__ F,
                                                      uint64_t *__restrict__ O, TsdfGrid g,
                                                      int W, Cols cl, int cj,
                                                      int32_t *__restrict__ changed,
                                                      const int32_t *__restrict__ skip)
{
    // a round enqueued after the labelling settled does nothing
    if (skip && *skip == 0) return;

    __shared__ uint64_t sA[kBlock], sB[kBlock], sT[kBlock];
    const int j = (int)threadIdx.x % cj, sg = (int)threadIdx.x / cj;
    const int64_t c = (int64_t)blockIdx.x * cj + j;
    const bool act = sg < cl.nseg && c < cl.ncols;
    const int64_t base = act ? col_base<AXIS>(c, g, W) : 0;
    const int r0 = sg * kSegRows;
    const int nr = !act ? 0 : (cl.rows - r0 < kSegRows ? cl.rows - r0 : kSegRows);
    uint64_t f[kSegRows], o[kSegRows], o0[kSegRows];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k) {
        f[k] = k < nr ? F[base + (int64_t)(r0 + k) * cl.stride] : 0ull;
        o[k] = k < nr ? O[base + (int64_t)(r0 + k) * cl.stride] : 0ull;
        o0[k] = o[k];
    }
    // summary: reach out of the end, out of the start, free throughout
    uint64_t r = 0, tr = ~0ull;
#pragma unroll
    for (int k = 0; k < kSegRows; ++k)
        if (k < nr) {
            r = f[k] & (r | o[k]);
            tr &= f[k];
        }
    uint64_t rb = 0;
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k)
        if (k < nr) rb = f[k] & (rb | o[k]);
    sA[threadIdx.x] = r;
    sB[threadIdx.x] = rb;
    sT[threadIdx.x] = tr;
    __syncthreads();
    // carries, in place of the summaries: threads 0 .. cj - 1 are column j
    // of segment 0
    if ((int)threadIdx.x < cj && c < cl.ncols) {
        uint64_t carry = ~0ull;                           // the frame before row 0
        for (int q = 0; q < cl.nseg; ++q) {
            const int i = q * cj + j;
            const uint64_t a = sA[i];
            sA[i] = carry;
            carry = a | (sT[i] & carry);
        }
        carry = ~0ull;                                    // the frame after the last row
        for (int q = cl.nseg - 1; q >= 0; --q) {
            const int i = q * cj + j;
            const uint64_t b = sB[i];
            sB[i] = carry;
            carry = b | (sT[i] & carry);
        }
    }
    __syncthreads();
    if (!act) return;
    r = sA[threadIdx.x];
#pragma unroll
    for (int k = 0; k < kSegRows; ++k)
        if (k < nr) {
            r = f[k] & (r | o[k]);
            o[k] = r;
        }
    r = sB[threadIdx.x];
#pragma unroll
    for (int k = kSegRows - 1; k >= 0; --k)
        if (k < nr) {
            r = f[k] & (r | o[k]);
            o[k] = r;
        }
    bool any = false;
#pragma unroll
    for (int k = 0; k < kSegRows; ++k)
        if (k < nr && o[k] != o0[k]) {
            O[base + (int64_t)(r0 + k) * cl.stride] = o[k];
            any = true;
        }
    if (any && *changed == 0) *changed = 1;
}

// ---- distance shells and phi -----------------------------------------------

// p = 0 on S_0 (a 6-neighbour with the other V~ value; outside the grid is
// 0), else 255 (not reached)
// bytes idx .. idx + 3 of p[0, n) (0 outside it), p 4-byte aligned: two
// aligned words where they lie inside the buffer, bytes near its ends
__device__ __forceinline__ uint32_t word_any(const uint8_t *__restrict__ p, int64_t idx, int64_t n)
{
    const int64_t a = idx & ~(int64_t)3;
    if (a >= 0 && a + 8 <= n) {
        const uint32_t lo = *reinterpret_cast<const uint32_t *>(p + a);
        const int sh = (int)(idx & 3);
        if (sh == 0) return lo;
        const uint32_t hi = *reinterpret_cast<const uint32_t *>(p + a + 4);
        return __builtin_amdgcn_alignbyte(hi, lo, (uint32_t)sh);
    }
    uint32_t w = 0;
    for (int j = 0; j < 4; ++j) {
        const int64_t q = idx + j;
        if (q >= 0 && q < n) w |= (uint32_t)p[q] << (8 * j);
    }
    return w;
}

// p = 0 on S_0 (a 6-neighbour with the other V~ value; outside the grid is
// 0), else 255 (not reached).  Four voxels per thread (V~ 4-byte aligned:
// word loads; p has the shell kernel's padding).
__global__ __launch_bounds__(kBlock) void k_shell0(const uint8_t *__restrict__ vt,
                                                   uint8_t *__restrict__ p, TsdfGrid g)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i0 >= g.n) return;
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const uint32_t c = word_any(vt, i0, g.n);
    const uint32_t xm = word_any(vt, i0 - 1, g.n), xp = word_any(vt, i0 + 1, g.n);
    const uint32_t ym = word_any(vt, i0 - g.nx, g.n), yp = word_any(vt, i0 + g.nx, g.n);
    const uint32_t zm = word_any(vt, i0 - sxy, g.n), zp = word_any(vt, i0 + sxy, g.n);
    int x, y, z;
    coords(i0, g, x, y, z);
    uint32_t out = 0;
    for (int j = 0; j < 4; ++j) {
        const uint32_t cj = byte_of(c, j);
        const bool edge = (x > 0 ? byte_of(xm, j) : 0u) != cj ||
                          (x < g.nx - 1 ? byte_of(xp, j) : 0u) != cj ||
                          (y > 0 ? byte_of(ym, j) : 0u) != cj ||
                          (y < g.ny - 1 ? byte_of(yp, j) : 0u) != cj ||
                          (z > 0 ? byte_of(zm, j) : 0u) != cj ||
                          (z < g.nz - 1 ? byte_of(zp, j) : 0u) != cj;
        out |= (edge ? 0u : 255u) << (8 * j);
        step_voxel(g, x, y, z);
    }
    *reinterpret_cast<uint32_t *>(p + i0) = out;
}

// the same, one voxel per thread (V~ not 4-byte aligned)
__global__ __launch_bounds__(kBlock) void k_shell0_1(const uint8_t *__restrict__ vt,
                                                     uint8_t *__restrict__ p, TsdfGrid g)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.n) return;
    int x, y, z;
    coords(i, g, x, y, z);
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const uint8_t c = vt[i];
    const uint8_t nb[6] = {x > 0 ? vt[i - 1] : (uint8_t)0, x < g.nx - 1 ? vt[i + 1] : (uint8_t)0,
                           y > 0 ? vt[i - g.nx] : (uint8_t)0,
                           y < g.ny - 1 ? vt[i + g.nx] : (uint8_t)0,
                           z > 0 ? vt[i - sxy] : (uint8_t)0, z < g.nz - 1 ? vt[i + sxy] : (uint8_t)0};
    bool edge = false;
    for (int k = 0; k < 6; ++k) edge |= nb[k] != c;
    p[i] = edge ? 0 : 255;
}

// Shell m: the unreached voxels (255) with a 6-neighbour in shell m - 1.
// Four voxels per thread as one aligned word: byte-wide loads, one per lane
// and neighbour, capped the one-voxel form at the rate the memory pipeline
// issues instructions.  Neighbour words at any byte offset are put together
// from two aligned words; `p` has kShellPad bytes of readable padding on
// both sides, so every load stays inside the buffer (bytes outside the grid
// are never used: the coordinate tests exclude them).  Voxels written in
// this pass go from 255 to m, neither of which is m - 1, so a neighbour
// read before or after the write gives the same answer; no two threads
// write the same word.

__global__ __launch_bounds__(kBlock) void k_shell(uint8_t *__restrict__ p, TsdfGrid g, int m)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i0 >= g.n) return;
    const uint32_t c = *reinterpret_cast<const uint32_t *>(p + i0);
    int live = 0;
    for (int j = 0; j < 4; ++j)
        if (i0 + j < g.n && byte_of(c, j) == 255u) live |= 1 << j;
    if (!live) return;
    const int64_t sxy = (int64_t)g.nx * g.ny;
    const uint32_t prev = (uint32_t)(m - 1);
    const uint32_t wl = *reinterpret_cast<const uint32_t *>(p + i0 - 4);
    const uint32_t wr = *reinterpret_cast<const uint32_t *>(p + i0 + 4);
    const uint32_t xm = __builtin_amdgcn_alignbyte(c, wl, 3u);   // bytes i0 - 1 + j
    const uint32_t xp = __builtin_amdgcn_alignbyte(wr, c, 1u);   // bytes i0 + 1 + j
    const uint32_t ym = word_at(p, i0 - g.nx), yp = word_at(p, i0 + g.nx);
    const uint32_t zm = word_at(p, i0 - sxy), zp = word_at(p, i0 + sxy);
    uint32_t out = c;
    for (int j = 0; j < 4; ++j) {
        if (!((live >> j) & 1)) continue;
        int x, y, z;
        coords(i0 + j, g, x, y, z);
        const bool hit = (x > 0 && byte_of(xm, j) == prev) ||
                         (x < g.nx - 1 && byte_of(xp, j) == prev) ||
                         (y > 0 && byte_of(ym, j) == prev) ||
                         (y < g.ny - 1 && byte_of(yp, j) == prev) ||
                         (z > 0 && byte_of(zm, j) == prev) ||
                         (z < g.nz - 1 && byte_of(zp, j) == prev);
        if (hit) out = (out & ~(0xffu << (8 * j))) | ((uint32_t)m << (8 * j));
    }
    if (out != c) *reinterpret_cast<uint32_t *>(p + i0) = out;
}

// S_0, the P <= 4 shells and phi in one pass over LDS tiles.  A block
// owns a 64 x 8 x 8 tile of voxels and loads V~ over it with a halo of
// P + 1 voxels in y and z and 8 in x (two LDS words: the tile's rows stay
// word aligned), then runs in LDS what the per-grid passes above do: S_0,
// then P shell steps, four voxels per 32-bit word with bytewise tests.
// The values of a step are correct wherever the previous step's were
// correct one voxel further in, so after P steps they are correct on the
// tile itself; voxels outside the grid read V~ = 0 and hold a p that never
// equals a shell index m - 1 < 4 and is never overwritten.  phi is written
// from the tile's p with the same operations as k_phi, so the results are
// the same bits; p never goes to memory.  V~ is 0 or 1 (the threshold
// pass's output).
constexpr int kShTX = 64, kShTY = 8, kShTZ = 8, kShHX = 8;

// 0xff in each byte of v that is zero, 0 elsewhere (exact, no carries
// between bytes)
__device__ __forceinline__ uint32_t zero_bytes(uint32_t v)
{
    uint32_t t = (v & 0x7f7f7f7fu) + 0x7f7f7f7fu;
    t = ~(t | v | 0x7f7f7f7fu);
    return (t >> 7) * 0xffu;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_shells_phi_tile(const uint8_t *__restrict__ vt,
                                                            const uint64_t *__restrict__ O,
                                                            float *__restrict__ phi, TsdfGrid g,
                                                            int W, float h, float r)
{
    static_assert(P >= 1 && P <= 4 && P + 1 <= kShHX, "tile halo");
    constexpr int H = P + 1;
    constexpr int LX = kShTX + 2 * kShHX, WX = LX / 4;
    constexpr int LY = kShTY + 2 * H, LZ = kShTZ + 2 * H;
    constexpr int NW = WX * LY * LZ, SY = WX, SZ = WX * LY;
    // one byte per voxel: V~ (0 or 1) in bit 7, p in bits 0..6 with 0x7f
    // for "not reached" (255 of the per-grid passes) and 0x7e outside the
    // grid; S_0 reads only bit 7 and writes only bits 0..6, so it runs in
    // place
    constexpr uint32_t kHi = 0x80808080u, kLo = 0x7f7f7f7fu;
    __shared__ uint32_t T[NW];
    // the outside word of each of the tile's rows (the tile's 64 columns
    // are one word), read here so that the phi pass at the end does not
    // wait on one load per row
    __shared__ uint64_t Ow[kShTY * kShTZ];
    const int x0 = (int)blockIdx.x * kShTX - kShHX;
    const int y0 = (int)blockIdx.y * kShTY - H, z0 = (int)blockIdx.z * kShTZ - H;
    if (threadIdx.x < kShTY * kShTZ) {
        const int gy = (int)blockIdx.y * kShTY + (int)threadIdx.x % kShTY;
        const int gz = (int)blockIdx.z * kShTZ + (int)threadIdx.x / kShTY;
        Ow[threadIdx.x] = gy < g.ny && gz < g.nz ? O[((int64_t)gz * g.ny + gy) * W + blockIdx.x] : 0ull;
    }
    for (int w = threadIdx.x; w < NW; w += kBlock) {
        const int wx = w % WX, t = w / WX, ly = t % LY, lz = t / LY;
        const int gx = x0 + 4 * wx, gy = y0 + ly, gz = z0 + lz;
        uint32_t v = 0x7e7e7e7eu;
        if (gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz) {
            const int64_t row = ((int64_t)gz * g.ny + gy) * g.nx;
            for (int j = 0; j < 4; ++j)
                if (gx + j >= 0 && gx + j < g.nx)
                    v = (v & ~(0xffu << (8 * j))) | ((vt[row + gx + j] ? 0x80u : 0x00u) << (8 * j));
        }
        T[w] = v;
    }
    __syncthreads();
    // interior words: every 6-neighbour of their voxels lies in the tile
    constexpr int IX = WX - 2, IY = LY - 2, IZ = LZ - 2;
    // a thread keeps one (word, row) column and walks it along z
    for (int q = threadIdx.x; q < IX * IY; q += kBlock) {
        int w = (LY + 1 + q / IX) * WX + 1 + q % IX;   // lz = 1
        for (int lz = 1; lz <= IZ; ++lz, w += SZ) {
            const uint32_t c = T[w];
            const uint32_t xm = __builtin_amdgcn_alignbyte(c, T[w - 1], 3u);
            const uint32_t xp = __builtin_amdgcn_alignbyte(T[w + 1], c, 1u);
            const uint32_t d = ((c ^ xm) | (c ^ xp) | (c ^ T[w - SY]) | (c ^ T[w + SY]) |
                                (c ^ T[w - SZ]) | (c ^ T[w + SZ])) & kHi;
            // in-grid bytes (low bits 0x7f after the load: 0x00 or 0x80 there)
            const uint32_t in = zero_bytes(c & kLo);
            const uint32_t p = zero_bytes(d) & kLo;   // 0x7f: no neighbour differs; 0: S_0
            T[w] = (c & kHi) | (p & in) | (0x7e7e7e7eu & ~in);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 1; m <= P; ++m) {
        const uint32_t prev = (uint32_t)(m - 1) * 0x01010101u;
        for (int q = threadIdx.x; q < IX * IY; q += kBlock) {
          int w = (LY + 1 + q / IX) * WX + 1 + q % IX;   // lz = 1
          for (int lz = 1; lz <= IZ; ++lz, w += SZ) {
            const uint32_t c = T[w];
            const uint32_t live = zero_bytes((c & kLo) ^ kLo);   // not reached yet
            if (!live) continue;
            const uint32_t xm = __builtin_amdgcn_alignbyte(c, T[w - 1], 3u);
            const uint32_t xp = __builtin_amdgcn_alignbyte(T[w + 1], c, 1u);
            const uint32_t hit = zero_bytes((xm & kLo) ^ prev) | zero_bytes((xp & kLo) ^ prev) |
                                 zero_bytes((T[w - SY] & kLo) ^ prev) |
                                 zero_bytes((T[w + SY] & kLo) ^ prev) |
                                 zero_bytes((T[w - SZ] & kLo) ^ prev) |
                                 zero_bytes((T[w + SZ] & kLo) ^ prev);
            const uint32_t set = live & hit & kLo;
            // 0x7f becomes m: a neighbour read before or after this store
            // sees a value other than m - 1 either way
            if (set) T[w] = (c & ~set) | (((uint32_t)m * 0x01010101u) & set);
          }
        }
        __syncthreads();
    }
    static_assert(kBlock % kShTX == 0, "whole rows per round");
    const int lx = (int)threadIdx.x % kShTX;
    const int gx = (int)blockIdx.x * kShTX + lx;
    for (int t = (int)threadIdx.x / kShTX; t < kShTY * kShTZ; t += kBlock / kShTX) {
        const int ly = t % kShTY, lz = t / kShTY;
        const int gy = (int)blockIdx.y * kShTY + ly, gz = (int)blockIdx.z * kShTZ + lz;
        if (gx >= g.nx || gy >= g.ny || gz >= g.nz) continue;
        const int cx = kShHX + lx;
        const uint32_t pj = byte_of(T[((H + lz) * LY + H + ly) * WX + (cx >> 2)], cx & 3) & 0x7fu;
        const int64_t row = (int64_t)gz * g.ny + gy;
        const bool out = (Ow[lz * kShTY + ly] >> (gx & 63)) & 1ull;   // gx >> 6 == blockIdx.x
        const float delta = pj == 0x7fu ? r : (float)pj * h;
        const float sg = out ? delta : -delta;
        phi[row * g.nx + gx] = fminf(fmaxf(sg, -r), r);
    }
}

// phi = clip(s p h, -r, r); s = +1 where the packed outside bit is set.
// Four voxels per thread (p padded and aligned); one float4 store when phi
// is 16-byte aligned.
__global__ __launch_bounds__(kBlock) void k_phi(const uint8_t *__restrict__ p,
                                                const uint64_t *__restrict__ O,
                                                float *__restrict__ phi, TsdfGrid g, int W,
                                                float h, float r, int vec)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i0 >= g.n) return;
    const uint32_t pw = *reinterpret_cast<const uint32_t *>(p + i0);
    int x, y, z;
    coords(i0, g, x, y, z);
    float f[4];
    for (int j = 0; j < 4; ++j) {
        const uint32_t pj = byte_of(pw, j);
        bool out = false;
        if (i0 + j < g.n) out = (O[((int64_t)z * g.ny + y) * W + (x >> 6)] >> (x & 63)) & 1ull;
        const float delta = pj == 255u ? r : (float)pj * h;
        const float sg = out ? delta : -delta;
        f[j] = fminf(fmaxf(sg, -r), r);
        step_voxel(g, x, y, z);
    }
    if (vec && i0 + 4 <= g.n) {
        *reinterpret_cast<float4 *>(phi + i0) = make_float4(f[0], f[1], f[2], f[3]);
    } else {
        for (int j = 0; i0 + j < g.n && j < 4; ++j) phi[i0 + j] = f[j];
    }
}

// ---- marching cubes --------------------------------------------------------
// Count pass, per lattice point: mask of crossed edges +x/+y/+z (bits 0..2)
// and the case of the cell it anchors (bit k set when corner k = (k & 1,
// k >> 1 & 1, k >> 2 & 1) is inside, phi < iso), one byte each; the vertex
// and triangle counts follow from them.
// Over 64 x 4 x 4 tiles: a block loads the inside bits of its tile plus
// one point further along each axis into LDS (each phi read once per tile,
// about 1.6x over the grid), then each thread takes four consecutive
// points of a row from LDS.  Points whose +x, +y or +z
// neighbour lies outside the grid never use it (the coordinate tests), so
// those LDS bytes are only placeholders.
constexpr int kMcTX = 64, kMcTY = 4, kMcTZ = 4;

__global__ __launch_bounds__(kBlock) void k_mc_count_tile(const float *__restrict__ phi,
                                                          TsdfGrid g, float iso,
                                                          uint8_t *__restrict__ mask,
                                                          uint8_t *__restrict__ cases)
{
    constexpr int LX = kMcTX + 1, LY = kMcTY + 1, LZ = kMcTZ + 1, NL = LX * LY * LZ;
    static_assert((kMcTX / 4) * kMcTY * kMcTZ == kBlock, "four points per thread");
    __shared__ uint8_t ins[NL];
    const int bx = (int)blockIdx.x * kMcTX, by = (int)blockIdx.y * kMcTY;
    const int bz = (int)blockIdx.z * kMcTZ;
    constexpr int PER = (NL + kBlock - 1) / kBlock;
    uint8_t v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = (int)threadIdx.x + k * kBlock;
        const int lx = q % LX, t = q / LX, ly = t % LY, lz = t / LY;
        const int gx = bx + lx, gy = by + ly, gz = bz + lz;
        // points outside the grid read point 0 and count as outside: no
        // branch between the loads, so all PER are in flight at once
        const bool ok = q < NL && gx < g.nx && gy < g.ny && gz < g.nz;
        const float f = phi[ok ? ((int64_t)gz * g.ny + gy) * g.nx + gx : 0];
        v[k] = ok && f < iso ? 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int q = (int)threadIdx.x + k * kBlock;
        if (q < NL) ins[q] = v[k];
    }
    __syncthreads();
    const int lx0 = ((int)threadIdx.x % (kMcTX / 4)) * 4;
    const int t = (int)threadIdx.x / (kMcTX / 4), ly = t % kMcTY, lz = t / kMcTY;
    const int gy = by + ly, gz = bz + lz;
    if (gy >= g.ny || gz >= g.nz) return;
    const int64_t row = ((int64_t)gz * g.ny + gy) * g.nx;
    for (int j = 0; j < 4; ++j) {
        const int lx = lx0 + j, gx = bx + lx;
        if (gx >= g.nx) break;
        const uint8_t *c = ins + (lz * LY + ly) * LX + lx;
        const int in = c[0];
        int m = 0;
        if (gx < g.nx - 1 && c[1] != in) m |= 1;
        if (gy < g.ny - 1 && c[LX] != in) m |= 2;
        if (gz < g.nz - 1 && c[LX * LY] != in) m |= 4;
        int cs = 0;
        if (gx < g.nx - 1 && gy < g.ny - 1 && gz < g.nz - 1) {
            // corner k = (k & 1, k >> 1 & 1, k >> 2 & 1)
#pragma unroll
            for (int k = 0; k < 8; ++k)
                cs |= (int)c[(k & 1) + ((k >> 1) & 1) * LX + ((k >> 2) & 1) * LX * LY] << k;
        }
        mask[row + gx] = (uint8_t)m;
        cases[row + gx] = (uint8_t)cs;
    }
}

// Gradient of phi at a lattice point along one axis, phi per voxel:
// central difference halved inside, one-sided on the first and last point,
// 0 on an axis of size 1.  The two reads are split from the arithmetic and
// made unconditional (the point itself where a neighbour is missing), so
// that the twelve reads of a vertex's two gradients are all in flight
// before the first is used.
__device__ __forceinline__ void lattice_reads(const float *__restrict__ phi, int64_t i, int c,
                                              int n, int64_t step, float &a, float &b)
{
    a = phi[c < n - 1 ? i + step : i];
    b = phi[c > 0 ? i - step : i];
}

// the same operations as the three cases: phi[i+1] - phi[i] at c = 0,
// phi[i] - phi[i-1] at c = n - 1, (phi[i+1] - phi[i-1]) / 2 between
__device__ __forceinline__ float lattice_diff(float a, float b, int c, int n)
{
    const float d = __fsub_rn(a, b);
    if (n < 2) return 0.0f;
    return (c == 0 || c == n - 1) ? d : __fmul_rn(d, 0.5f);
}

// The vertex on edge `a` (0: +x, 1: +y, 2: +z) of lattice point i, into
// slot v: the crossing of iso by linear interpolation along the edge, and
// with normals the normalised interpolation of the lattice gradients at the
// edge's ends.
__device__ __forceinline__ void mc_emit_vertex(const float *__restrict__ phi, const TsdfGrid &g,
                                               float iso, float *__restrict__ verts,
                                               float *__restrict__ normals, int64_t i, int a,
                                               uint32_t v)
{
    int x, y, z;
    coords(i, g, x, y, z);
    const float c0 = (float)(g.o[0] + ((double)x + 0.5) * g.h);
    const float c1 = (float)(g.o[1] + ((double)y + 0.5) * g.h);
    const float c2 = (float)(g.o[2] + ((double)z + 0.5) * g.h);
    const int64_t sx = g.nx, sxy = (int64_t)g.nx * g.ny;
    const int64_t step = a == 0 ? 1 : (a == 1 ? sx : sxy);
    const float fa = phi[i], fb = phi[i + step];
    // gradient reads at both ends of the edge, issued before any is used
    const int xb = x + (a == 0), yb = y + (a == 1), zb = z + (a == 2);
    float r[12];
    if (normals) {
        lattice_reads(phi, i, x, g.nx, 1, r[0], r[1]);
        lattice_reads(phi, i, y, g.ny, sx, r[2], r[3]);
        lattice_reads(phi, i, z, g.nz, sxy, r[4], r[5]);
        lattice_reads(phi, i + step, xb, g.nx, 1, r[6], r[7]);
        lattice_reads(phi, i + step, yb, g.ny, sx, r[8], r[9]);
        lattice_reads(phi, i + step, zb, g.nz, sxy, r[10], r[11]);
    }
    const float t = __fdiv_rn(iso - fa, fb - fa);
    const float pa = __fadd_rn(a == 0 ? c0 : (a == 1 ? c1 : c2), __fmul_rn(t, g.hf));
    verts[3 * (int64_t)v + 0] = a == 0 ? pa : c0;
    verts[3 * (int64_t)v + 1] = a == 1 ? pa : c1;
    verts[3 * (int64_t)v + 2] = a == 2 ? pa : c2;
    if (normals) {
        // n = (1 - t) g_a + t g_b, normalised; float32, one rounded
        // operation at a time
        const float ga[3] = {lattice_diff(r[0], r[1], x, g.nx), lattice_diff(r[2], r[3], y, g.ny),
                             lattice_diff(r[4], r[5], z, g.nz)};
        const float gb[3] = {lattice_diff(r[6], r[7], xb, g.nx),
                             lattice_diff(r[8], r[9], yb, g.ny),
                             lattice_diff(r[10], r[11], zb, g.nz)};
        const float w = __fsub_rn(1.0f, t);
        float nv[3];
        for (int k = 0; k < 3; ++k)
            nv[k] = __fadd_rn(__fmul_rn(w, ga[k]), __fmul_rn(t, gb[k]));
        const float l2 = __fadd_rn(__fadd_rn(__fmul_rn(nv[0], nv[0]), __fmul_rn(nv[1], nv[1])),
                                   __fmul_rn(nv[2], nv[2]));
        // correctly rounded float32 square root: the FP64 root rounded to
        // float32 (53 >= 2 * 24 + 2 bits, so the double rounding is exact);
        // v_sqrt_f32 alone is not exact
        const float l = (float)sqrt((double)l2);
        for (int k = 0; k < 3; ++k)
            normals[3 * (int64_t)v + k] = l > 0.0f ? __fdiv_rn(nv[k], l) : 0.0f;
    }
}

// Triangle k of the cell at lattice point i (case cs), into slot t: its
// corners are the vertices of the cell edges the case table names; a point
// q's first vertex is voff[q] (its offset within its scan tile) +
// vbase[q / kScanTile], and its edges' vertices follow in axis order.
__device__ __forceinline__ void mc_emit_tri(const TsdfGrid &g, const int8_t *__restrict__ tris_of,
                                            const uint8_t *__restrict__ mask,
                                            const uint16_t *__restrict__ voff,
                                            const uint32_t *__restrict__ vbase,
                                            int32_t *__restrict__ tris, int64_t i, int cs, int k,
                                            uint32_t t)
{
    const int64_t sx = g.nx, sxy = (int64_t)g.nx * g.ny;
    for (int e = 0; e < 3; ++e) {
        const int edge = tris_of[cs * 15 + 3 * k + e];
        // edges are numbered (axis, lower corner): 4 per axis
        const int axis = edge >> 2, nth = edge & 3;
        // the nth corner (ascending) whose bit `axis` is clear
        const int lo = nth & ((1 << axis) - 1);
        const int corner = ((nth >> axis) << (axis + 1)) | lo;
        const int64_t q = i + ((corner & 1) ? 1 : 0) + ((corner & 2) ? sx : 0) +
                          ((corner & 4) ? sxy : 0);
        const int mq = mask[q];
        const uint32_t id = (uint32_t)voff[q] + vbase[q / kScanTile] +
                            (uint32_t)__popc(mq & ((1 << axis) - 1));
        tris[3 * (int64_t)t + e] = (int32_t)id;
    }
}

__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t ws[kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < kBlock / 64; ++k) {
        if (k < w) off += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// One block per scan tile.  Points with a vertex or a triangle are a small
// share of the grid and need different amounts of work (0 to 3 vertices, 0
// to 5 triangles), so the block lists the tile's vertices, then its
// triangles, as items in LDS, in slot order (the slots come from an
// in-block scan of the per-point counts, the same offsets the count pass
// stored), and each thread emits one item at a time: every lane runs the
// same code on every item.
__global__ __launch_bounds__(kBlock) void k_mc_emit(const float *__restrict__ phi, TsdfGrid g,
                                                    float iso, const uint8_t *__restrict__ ntri,
                                                    const int8_t *__restrict__ tris_of,
                                                    const uint8_t *__restrict__ mask,
                                                    const uint8_t *__restrict__ cases,
                                                    const uint16_t *__restrict__ voff,
                                                    const uint32_t *__restrict__ vbase,
                                                    const uint32_t *__restrict__ tbase,
                                                    float *__restrict__ verts,
                                                    int32_t *__restrict__ tris,
                                                    float *__restrict__ normals)
{
    static_assert(kScanItems == 4, "one word of mask and case bytes per thread");
    static_assert(kScanTile == 1024, "item packing: point in tile in bits 0..9");
    __shared__ uint8_t nt_lds[256];
    // vertex items (point | axis << 10), then triangle items (point |
    // k << 10 | case << 13): at most 3 and 5 per point
    __shared__ uint32_t items[5 * kScanTile];
    // the case table's triangle edges (256 x 15 bytes, word aligned), read
    // from LDS by the triangle items
    __shared__ uint32_t tri_lds[256 * 15 / 4];
    nt_lds[threadIdx.x] = ntri[threadIdx.x];              // kBlock == 256 cases
    for (int k = threadIdx.x; k < 256 * 15 / 4; k += kBlock)
        tri_lds[k] = reinterpret_cast<const uint32_t *>(tris_of)[k];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int64_t p0 = base + (int64_t)threadIdx.x * kScanItems;
    uint32_t mw = 0, cw = 0;
    if (p0 + 4 <= g.n) {                                  // p0 is a multiple of 4
        mw = *reinterpret_cast<const uint32_t *>(mask + p0);
        cw = *reinterpret_cast<const uint32_t *>(cases + p0);
    } else {
        for (int k = 0; p0 + k < g.n && k < 4; ++k) {
            mw |= (uint32_t)mask[p0 + k] << (8 * k);
            cw |= (uint32_t)cases[p0 + k] << (8 * k);
        }
    }
    uint32_t tc[kScanItems], sv = 0, st = 0;
    for (int k = 0; k < kScanItems; ++k) {
        tc[k] = p0 + k < g.n ? (uint32_t)nt_lds[(cw >> (8 * k)) & 0xffu] : 0u;
        st += tc[k];
        sv += (uint32_t)__popc((mw >> (8 * k)) & 7u);
    }
    // both counts in one scan: a tile has at most 3072 vertices, so they
    // stay in the low 16 bits
    uint32_t tot;
    const uint32_t r = block_scan_excl(sv | (st << 16), &tot);
    const uint32_t nv = tot & 0xffffu, ntr = tot >> 16;
    uint32_t rv = r & 0xffffu, rt = r >> 16;
    const uint32_t lp = threadIdx.x * kScanItems;
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t m = (mw >> (8 * k)) & 7u;
        for (int a = 0; a < 3; ++a)
            if ((m >> a) & 1u) items[rv++] = (lp + k) | ((uint32_t)a << 10);
    }
    __syncthreads();
    const uint32_t vb = vbase[blockIdx.x], tb = tbase[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < nv; j += kBlock) {
        const uint32_t e = items[j];
        mc_emit_vertex(phi, g, iso, verts, normals, base + (e & 1023u), (int)(e >> 10), vb + j);
    }
    __syncthreads();
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t cs = (cw >> (8 * k)) & 0xffu;
        for (uint32_t q = 0; q < tc[k]; ++q) items[rt++] = (lp + k) | (q << 10) | (cs << 13);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < ntr; j += kBlock) {
        const uint32_t e = items[j];
        mc_emit_tri(g, reinterpret_cast<const int8_t *>(tri_lds), mask, voff, vbase, tris,
                    base + (e & 1023u), (int)(e >> 13),
                    (int)((e >> 10) & 7u), tb + j);
    }
}

// ---- exclusive scan of uint32 (three kernels) ------------------------------

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const uint32_t *__restrict__ in,
                                                       uint32_t *__restrict__ out, int64_t n,
                                                       uint32_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems], s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_scan_excl(s, &tot);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Marching-cubes scan tiles: the vertex count (edges set in the mask) and
// the triangle count (of the cell's case) of each point are formed here
// from the count pass's two bytes; each point gets its vertex offset within
// the tile, and the tile its two totals (the emit pass scans the triangle
// counts of its tile again, since only the point itself needs them).
__global__ __launch_bounds__(kBlock) void k_mc_scan_tiles(const uint8_t *__restrict__ mask,
                                                          const uint8_t *__restrict__ cases,
                                                          const uint8_t *__restrict__ ntri,
                                                          int64_t n, uint16_t *__restrict__ voff,
                                                          uint32_t *__restrict__ vsums,
                                                          uint32_t *__restrict__ tsums)
{
    static_assert(kScanItems == 4, "one word of mask and case bytes per thread");
    __shared__ uint8_t nt_lds[256];
    nt_lds[threadIdx.x] = ntri[threadIdx.x];              // kBlock == 256 cases
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t mw = 0, cw = 0;
    if (base + 4 <= n) {                                  // base is a multiple of 4
        mw = *reinterpret_cast<const uint32_t *>(mask + base);
        cw = *reinterpret_cast<const uint32_t *>(cases + base);
    } else {
        for (int k = 0; base + k < n && k < 4; ++k) {
            mw |= (uint32_t)mask[base + k] << (8 * k);
            cw |= (uint32_t)cases[base + k] << (8 * k);
        }
    }
    uint32_t vc[kScanItems], sv = 0, st = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const bool in = base + k < n;
        vc[k] = in ? (uint32_t)__popc((mw >> (8 * k)) & 0xffu) : 0u;
        st += in ? (uint32_t)nt_lds[(cw >> (8 * k)) & 0xffu] : 0u;
        sv += vc[k];
    }
    // both totals in one scan: a tile has at most 3 * kScanTile = 3072
    // vertices, so they stay in the low 16 bits (and a point's offset
    // within its tile fits a u16)
    static_assert(3 * kScanTile < (1 << 16), "tile vertex offsets in 16 bits");
    uint32_t tot;
    uint32_t rv = block_scan_excl(sv | (st << 16), &tot) & 0xffffu;
    uint16_t o[kScanItems];
    for (int k = 0; k < kScanItems; ++k) {
        o[k] = (uint16_t)rv;
        rv += vc[k];
    }
    if (base + 4 <= n) {                                  // 8-byte aligned: base % 4 == 0
        *reinterpret_cast<uint2 *>(voff + base) =
            make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16));
    } else {
        for (int k = 0; base + k < n && k < 4; ++k) voff[base + k] = o[k];
    }
    if (threadIdx.x == 0) {
        vsums[blockIdx.x] = tot & 0xffffu;
        tsums[blockIdx.x] = tot >> 16;
    }
}

// One 1024-thread block: exclusive scans of the vertex and the triangle
// tile totals in place, grand totals after them.
constexpr int kSums2Block = 1024;

__device__ __forceinline__ uint32_t block_scan_excl_1024(uint32_t v, uint32_t *total,
                                                         uint32_t *ws)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int k = 0; k < kSums2Block / 64; ++k) {
        if (k < w) off += ws[k];
        tot += ws[k];
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// Chunks of kSums2Chunk entries of both arrays go through LDS: loaded and
// stored coalesced, scanned there with eight consecutive entries per
// thread (one block on one CU: per-thread contiguous global reads were
// uncoalesced and took 95 us for 32k tiles).
constexpr int kSums2Chunk = kSums2Block * 8;

__global__ __launch_bounds__(kSums2Block) void k_scan_sums2(uint32_t *__restrict__ a,
                                                            uint32_t *__restrict__ b, int nb)
{
    __shared__ uint32_t la[kSums2Chunk], lb[kSums2Chunk];
    __shared__ uint32_t ws[kSums2Block / 64];
    uint32_t carry_a = 0, carry_b = 0;
    for (int c0 = 0; c0 < nb; c0 += kSums2Chunk) {
        const int m = nb - c0 < kSums2Chunk ? nb - c0 : kSums2Chunk;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = k * kSums2Block + (int)threadIdx.x;
            la[i] = i < m ? a[c0 + i] : 0u;
            lb[i] = i < m ? b[c0 + i] : 0u;
        }
        __syncthreads();
        uint32_t va[8], vb[8], sa = 0, sb = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            va[k] = la[8 * threadIdx.x + k];
            vb[k] = lb[8 * threadIdx.x + k];
            sa += va[k];
            sb += vb[k];
        }
        uint32_t ta, tb;
        uint32_t ra = carry_a + block_scan_excl_1024(sa, &ta, ws);
        uint32_t rb = carry_b + block_scan_excl_1024(sb, &tb, ws);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            la[8 * threadIdx.x + k] = ra;
            lb[8 * threadIdx.x + k] = rb;
            ra += va[k];
            rb += vb[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = k * kSums2Block + (int)threadIdx.x;
            if (i < m) {
                a[c0 + i] = la[i];
                b[c0 + i] = lb[i];
            }
        }
        carry_a += ta;
        carry_b += tb;
        __syncthreads();   // la / lb are refilled by the next chunk
    }
    if (threadIdx.x == 0) {
        a[nb] = carry_a;
        b[nb] = carry_b;
    }
}

// one block: exclusive scan of the tile sums in place, grand total after
// them.  Each thread owns a contiguous chunk (sum it, one block scan of the
// chunk totals, then write the chunk's prefixes): walking 256 sums per
// block-wide step took 35 us for 32k tiles.
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint32_t *__restrict__ sums, int nb)
{
    const int per = (nb + kBlock - 1) / kBlock;
    const int lo = (int)threadIdx.x * per;
    const int hi = lo + per < nb ? lo + per : nb;
    // chunks are read and written 16 entries at a time so that the loads
    // of a group are in flight together
    uint32_t s = 0;
    for (int i0 = lo; i0 < hi; i0 += 16) {
        uint32_t v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = i0 + k < hi ? sums[i0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < 16; ++k) s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_scan_excl(s, &tot);
    for (int i0 = lo; i0 < hi; i0 += 16) {
        uint32_t v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = i0 + k < hi ? sums[i0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (i0 + k < hi) sums[i0 + k] = run;
            run += v[k];
        }
    }
    if (threadIdx.x == 0) sums[nb] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(uint32_t *__restrict__ out, int64_t n,
                                                     const uint32_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const uint32_t add = sums[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kBlock)
        if (base + k < n) out[base + k] += add;
}

// ---- the case table (host) -------------------------------------------------
// Corner k of a cell is (k & 1, k >> 1 & 1, k >> 2 & 1); edge e = 4 axis + j
// joins the j-th corner (ascending) with bit `axis` clear to that corner plus
// the unit step along `axis`.
struct Table {
    uint8_t count[256];
    int8_t tri[256][15];
};

void make_table(Table &t)
{
    int ea[12], eb[12];
    int edge_of[8][8];
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) edge_of[a][b] = -1;
    int ne = 0;
    for (int axis = 0; axis < 3; ++axis)
        for (int a = 0; a < 8; ++a)
            if (!((a >> axis) & 1)) {
                ea[ne] = a;
                eb[ne] = a | (1 << axis);
                edge_of[a][eb[ne]] = edge_of[eb[ne]][a] = ne;
                ++ne;
            }
    // faces: corners counter-clockwise about the outward normal
    int face[6][4];
    int nf = 0;
    for (int axis = 0; axis < 3; ++axis) {
        const int u = (axis + 1) % 3, v = (axis + 2) % 3;
        for (int side = 0; side < 2; ++side) {
            const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};   // about +axis
            for (int k = 0; k < 4; ++k) {
                const int kk = side ? k : 3 - k;                     // -axis: reversed
                const int cu = uv[kk][0], cv = uv[kk][1];
                face[nf][k] = (side << axis) | (cu << u) | (cv << v);
            }
            ++nf;
        }
    }
    unsigned efaces[12] = {0};
    for (int f = 0; f < 6; ++f)
        for (int k = 0; k < 4; ++k) efaces[edge_of[face[f][k]][face[f][(k + 1) % 4]]] |= 1u << f;
    (void)ea;
    (void)eb;
    for (int cs = 0; cs < 256; ++cs) {
        int succ[12];
        for (int e = 0; e < 12; ++e) succ[e] = -1;
        for (int f = 0; f < 6; ++f) {
            int ce[4], cin[4], nc = 0;   // crossings in walk order; cin = outside->inside
            for (int k = 0; k < 4; ++k) {
                const int a = face[f][k], b = face[f][(k + 1) % 4];
                const int ia = (cs >> a) & 1, ib = (cs >> b) & 1;
                if (ia != ib) {
                    ce[nc] = edge_of[a][b];
                    cin[nc] = ib;
                    ++nc;
                }
            }
            for (int j = 0; j < nc; ++j) {
                if (!cin[j]) continue;
                for (int s = 1; s < nc; ++s) {
                    const int q = (j + s) % nc;
                    if (!cin[q]) {
                        succ[ce[j]] = ce[q];
                        break;
                    }
                }
            }
        }
        int n = 0;
        bool seen[12] = {false};
        for (int e0 = 0; e0 < 12; ++e0) {
            if (succ[e0] < 0 || seen[e0]) continue;
            int loop[12], k = 0;
            int e = e0;
            do {
                loop[k++] = e;
                seen[e] = true;
                e = succ[e];
            } while (e != e0);
            // fan apex: first vertex whose diagonals join edges sharing no face
            int apex = 0;
            for (int j = 0; j < k; ++j) {
                bool ok = true;
                for (int q = 0; q < k && ok; ++q) {
                    if (q == j || q == (j + 1) % k || q == (j + k - 1) % k) continue;
                    if (efaces[loop[j]] & efaces[loop[q]]) ok = false;
                }
                if (ok) {
                    apex = j;
                    break;
                }
            }
            for (int q = 1; q + 1 < k; ++q) {
                t.tri[cs][3 * n + 0] = (int8_t)loop[apex];
                t.tri[cs][3 * n + 1] = (int8_t)loop[(apex + q) % k];
                t.tri[cs][3 * n + 2] = (int8_t)loop[(apex + q + 1) % k];
                ++n;
            }
        }
        t.count[cs] = (uint8_t)n;
        for (int q = 3 * n; q < 15; ++q) t.tri[cs][q] = -1;
    }
}

const Table &table()
{
    static Table t;
    static std::once_flag once;
    std::call_once(once, [] { make_table(t); });
    return t;
}

hipError_t scan_launch(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *sums,
                       hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, sums, (int)nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, out, n, sums);
    return hipGetLastError();
}

}  // namespace

void mc_table_copy(uint8_t *count, int8_t *tri)
{
    const Table &t = table();
    for (int c = 0; c < 256; ++c) {
        count[c] = t.count[c];
        for (int q = 0; q < 15; ++q) tri[15 * c + q] = t.tri[c][q];
    }
}

int64_t mc_scan_sums_len(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// padding of the fast path's intermediates: three taps plus two words
static int64_t smooth_pad_a(const TsdfGrid &g)
{
    return ((int64_t)kFastSmooth * g.nx + 8 + 3) & ~(int64_t)3;
}

static int64_t smooth_pad_b(const TsdfGrid &g)
{
    return (2 * (int64_t)kFastSmooth * g.nx * g.ny + 16 + 7) & ~(int64_t)7;
}

size_t tsdf_smooth_a_bytes(const TsdfGrid &g)
{
    const int64_t fast = g.n + 2 * smooth_pad_a(g) + 8, wide = 4 * g.n;
    return (size_t)(fast > wide ? fast : wide);
}

size_t tsdf_smooth_b_bytes(const TsdfGrid &g)
{
    const int64_t fast = 2 * g.n + 2 * smooth_pad_b(g) + 16, wide = 8 * g.n;
    return (size_t)(fast > wide ? fast : wide);
}

hipError_t tsdf_smooth_launch(const uint8_t *surf, void *abuf, void *bbuf, uint8_t *vt,
                              const TsdfGrid &g, const Binomial &w, uint64_t thr, hipStream_t s)
{
    const bool fast = w.n <= kFastSmooth && ((uintptr_t)surf & 3) == 0 &&
                      ((uintptr_t)vt & 3) == 0;
    if (fast) {
        uint8_t *a8 = static_cast<uint8_t *>(abuf) + smooth_pad_a(g);
        uint8_t *b8 = static_cast<uint8_t *>(bbuf) + smooth_pad_b(g);
        const unsigned grid4 = grid_for((g.n + 3) / 4, kBlock);
        hipLaunchKernelGGL(k_smooth_x4, dim3(grid4), dim3(kBlock), 0, s, surf, a8, g, w);
        hipLaunchKernelGGL(k_smooth_y4, dim3(grid4), dim3(kBlock), 0, s, a8,
                           reinterpret_cast<uint16_t *>(b8), g, w);
        hipLaunchKernelGGL(k_smooth_z4, dim3(grid4), dim3(kBlock), 0, s, b8, vt, g, w, thr);
        return hipGetLastError();
    }
    uint32_t *a = static_cast<uint32_t *>(abuf);
    uint64_t *b = static_cast<uint64_t *>(bbuf);
    const unsigned grid = grid_for(g.n, kBlock);
    hipLaunchKernelGGL(k_smooth_x, dim3(grid), dim3(kBlock), 0, s, surf, a, g, w);
    hipLaunchKernelGGL(k_smooth_y, dim3(grid), dim3(kBlock), 0, s, a, b, g, w);
    hipLaunchKernelGGL(k_smooth_z, dim3(grid), dim3(kBlock), 0, s, b, vt, g, w, thr);
    return hipGetLastError();
}

hipError_t tsdf_smooth_sums_launch(const uint8_t *surf, void *abuf, void *bbuf, uint64_t *sums,
                                   const TsdfGrid &g, const Binomial &w, hipStream_t s)
{
    uint32_t *a = static_cast<uint32_t *>(abuf);
    uint64_t *b = static_cast<uint64_t *>(bbuf);
    const unsigned grid = grid_for(g.n, kBlock);
    hipLaunchKernelGGL(k_smooth_x, dim3(grid), dim3(kBlock), 0, s, surf, a, g, w);
    hipLaunchKernelGGL(k_smooth_y, dim3(grid), dim3(kBlock), 0, s, a, b, g, w);
    hipLaunchKernelGGL(k_smooth_z_sum, dim3(grid), dim3(kBlock), 0, s, b, sums, g, w);
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void k_stride_gather(const float *__restrict__ phi, TsdfGrid g,
                                                          int step, int mx, int my, int64_t m,
                                                          float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int64_t x = i % mx, yz = i / mx;
    const int64_t y = yz % my, z = yz / my;
    out[i] = phi[((z * step) * g.ny + y * step) * (int64_t)g.nx + x * step];
}

hipError_t mc_stride_gather_launch(const float *phi, const TsdfGrid &g, int step, int mx, int my,
                                   int mz, float *out, hipStream_t s)
{
    const int64_t m = (int64_t)mx * my * mz;
    hipLaunchKernelGGL(k_stride_gather, dim3(grid_for(m, kBlock)), dim3(kBlock), 0, s, phi, g,
                       step, mx, my, m, out);
    return hipGetLastError();
}

hipError_t tsdf_threshold_launch(const uint64_t *sums, const uint64_t *thr, uint8_t *vt,
                                 int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_threshold_sums, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, sums,
                       thr, vt, n);
    return hipGetLastError();
}

int tsdf_words_per_row(const TsdfGrid &g) { return (g.nx + 63) / 64; }

static Cols cols_of(const TsdfGrid &g, int axis)
{
    const int W = tsdf_words_per_row(g);
    Cols c;
    c.rows = axis == 1 ? g.ny : g.nz;
    c.ncols = (int64_t)W * (axis == 1 ? g.nz : g.ny);
    c.stride = axis == 1 ? W : (int64_t)W * g.ny;
    c.nseg = (c.rows + kSegRows - 1) / kSegRows;
    return c;
}

int64_t tsdf_seg_words(const TsdfGrid &g)
{
    const Cols a = cols_of(g, 1), b = cols_of(g, 2);
    const int64_t na = a.ncols * a.nseg, nb = b.ncols * b.nseg;
    return na > nb ? na : nb;
}

bool tsdf_smooth_pack_fused(const Binomial &w) { return w.n >= 1 && w.n <= 3; }

hipError_t tsdf_smooth_pack_launch(const uint8_t *surf, uint8_t *vt, uint64_t *F, uint64_t *O,
                                   const TsdfGrid &g, const Binomial &w, uint64_t thr,
                                   hipStream_t s)
{
    const dim3 tiles((unsigned)((g.nx + kSmTX - 1) / kSmTX), (unsigned)((g.ny + kSmTY - 1) / kSmTY),
                     (unsigned)((g.nz + kSmTZ - 1) / kSmTZ));
    const int W = tsdf_words_per_row(g);
    switch (w.n) {
    case 1: hipLaunchKernelGGL(k_smooth_pack_tile<1>, tiles, dim3(kBlock), 0, s, surf, vt, g, w, thr, W, F, O); break;
    case 2: hipLaunchKernelGGL(k_smooth_pack_tile<2>, tiles, dim3(kBlock), 0, s, surf, vt, g, w, thr, W, F, O); break;
    case 3: hipLaunchKernelGGL(k_smooth_pack_tile<3>, tiles, dim3(kBlock), 0, s, surf, vt, g, w, thr, W, F, O); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t tsdf_pack_launch(const uint8_t *vt, uint64_t *F, uint64_t *O, const TsdfGrid &g,
                            hipStream_t s)
{
    const int W = tsdf_words_per_row(g);
    const int64_t nw = (int64_t)W * g.ny * g.nz;
    hipLaunchKernelGGL(k_pack_free, dim3(grid_for(nw, kBlock / 64)), dim3(kBlock), 0, s, vt, g, W,
                       F, O);
    return hipGetLastError();
}

hipError_t tsdf_flood_round_launch(const uint64_t *F, uint64_t *O, uint64_t *seg,
                                   const TsdfGrid &g, const int32_t *prev, int32_t *changed,
                                   hipStream_t s)
{
    const int W = tsdf_words_per_row(g);
    hipLaunchKernelGGL(k_sweep_x, dim3(grid_for((int64_t)g.ny * g.nz, kBlock)), dim3(kBlock), 0, s,
                       F, O, g, W, changed, prev);
    const int64_t ns = tsdf_seg_words(g);
    uint64_t *A = seg, *B = seg + ns, *T = seg + 2 * ns, *C = seg + 3 * ns, *D = seg + 4 * ns;
    for (int axis = 1; axis <= 2; ++axis) {
        const Cols cl = cols_of(g, axis);
        if (cl.nseg <= kFusedSegs) {
            const int cj = (kBlock / cl.nseg) & ~7;       // >= 8: whole 64-byte rows of words
            const unsigned gb = (unsigned)((cl.ncols + cj - 1) / cj);
            if (axis == 1)
                hipLaunchKernelGGL(k_seg_fused<1>, dim3(gb), dim3(kBlock), 0, s, F, O, g, W, cl,
                                   cj, changed, prev);
            else
                hipLaunchKernelGGL(k_seg_fused<2>, dim3(gb), dim3(kBlock), 0, s, F, O, g, W, cl,
                                   cj, changed, prev);
            continue;
        }
        const unsigned gs = grid_for(cl.ncols * cl.nseg, kBlock);
        if (axis == 1)
            hipLaunchKernelGGL(k_seg_summary<1>, dim3(gs), dim3(kBlock), 0, s, F, O, g, W, cl, A, B,
                               T, prev);
        else
            hipLaunchKernelGGL(k_seg_summary<2>, dim3(gs), dim3(kBlock), 0, s, F, O, g, W, cl, A, B,
                               T, prev);
        hipLaunchKernelGGL(k_seg_carry, dim3(grid_for(cl.ncols, kBlock)), dim3(kBlock), 0, s, A, B,
                           T, cl, C, D, prev);
        if (axis == 1)
            hipLaunchKernelGGL(k_seg_apply<1>, dim3(gs), dim3(kBlock), 0, s, F, O, g, W, cl, C, D,
                               changed, prev);
        else
            hipLaunchKernelGGL(k_seg_apply<2>, dim3(gs), dim3(kBlock), 0, s, F, O, g, W, cl, C, D,
                               changed, prev);
    }
    return hipGetLastError();
}

// one z-layer plus two words, rounded up to a word: the farthest neighbour
// word of the four-voxel shell kernel
int64_t tsdf_shell_pad(const TsdfGrid &g) { return (((int64_t)g.nx * g.ny + 8) + 3) & ~(int64_t)3; }

hipError_t tsdf_shells_phi_launch(const uint8_t *vt, const uint64_t *O, uint8_t *p, float *phi,
                                  const TsdfGrid &g, int shells, float h, float r, hipStream_t s)
{
    if (shells >= 1 && shells <= 4) {
        const dim3 tiles((unsigned)((g.nx + kShTX - 1) / kShTX), (unsigned)((g.ny + kShTY - 1) / kShTY),
                         (unsigned)((g.nz + kShTZ - 1) / kShTZ));
        const int W = tsdf_words_per_row(g);
        switch (shells) {
        case 1: hipLaunchKernelGGL(k_shells_phi_tile<1>, tiles, dim3(kBlock), 0, s, vt, O, phi, g, W, h, r); break;
        case 2: hipLaunchKernelGGL(k_shells_phi_tile<2>, tiles, dim3(kBlock), 0, s, vt, O, phi, g, W, h, r); break;
        case 3: hipLaunchKernelGGL(k_shells_phi_tile<3>, tiles, dim3(kBlock), 0, s, vt, O, phi, g, W, h, r); break;
        default: hipLaunchKernelGGL(k_shells_phi_tile<4>, tiles, dim3(kBlock), 0, s, vt, O, phi, g, W, h, r); break;
        }
        return hipGetLastError();
    }
    const unsigned grid = grid_for(g.n, kBlock);
    const unsigned grid4 = grid_for((g.n + 3) / 4, kBlock);
    if (((uintptr_t)vt & 3) == 0)
        hipLaunchKernelGGL(k_shell0, dim3(grid4), dim3(kBlock), 0, s, vt, p, g);
    else
        hipLaunchKernelGGL(k_shell0_1, dim3(grid), dim3(kBlock), 0, s, vt, p, g);
    for (int m = 1; m <= shells; ++m)
        hipLaunchKernelGGL(k_shell, dim3(grid4), dim3(kBlock), 0, s, p, g, m);
    hipLaunchKernelGGL(k_phi, dim3(grid4), dim3(kBlock), 0, s, p, O, phi, g, tsdf_words_per_row(g),
                       h, r, ((uintptr_t)phi & 15) == 0 ? 1 : 0);
    return hipGetLastError();
}

hipError_t mc_count_launch(const float *phi, const TsdfGrid &g, float iso, const uint8_t *ntri,
                           uint8_t *mask, uint8_t *cases, uint16_t *voff, uint32_t *vsums,
                           uint32_t *tsums, hipStream_t s)
{
    const dim3 tiles((unsigned)((g.nx + kMcTX - 1) / kMcTX), (unsigned)((g.ny + kMcTY - 1) / kMcTY),
                     (unsigned)((g.nz + kMcTZ - 1) / kMcTZ));
    hipLaunchKernelGGL(k_mc_count_tile, tiles, dim3(kBlock), 0, s, phi, g, iso, mask, cases);
    const int64_t nb = (g.n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_mc_scan_tiles, dim3((unsigned)nb), dim3(kBlock), 0, s, mask, cases, ntri,
                       g.n, voff, vsums, tsums);
    hipLaunchKernelGGL(k_scan_sums2, dim3(1), dim3(kSums2Block), 0, s, vsums, tsums, (int)nb);
    return hipGetLastError();
}

hipError_t mc_emit_launch(const float *phi, const TsdfGrid &g, float iso, const uint8_t *ntri,
                          const int8_t *tris_of, const uint8_t *mask, const uint8_t *cases,
                          const uint16_t *voff, const uint32_t *vsums, const uint32_t *tsums,
                          float *verts, int32_t *tris, float *normals, hipStream_t s)
{
    hipLaunchKernelGGL(k_mc_emit, dim3(grid_for(g.n, kScanTile)), dim3(kBlock), 0, s, phi, g, iso,
                       ntri, tris_of, mask, cases, voff, vsums, tsums, verts, tris, normals);
    return hipGetLastError();
}

hipError_t scan_u32_launch(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *sums,
                           hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    return scan_launch(in, out, n, sums, s);
}
