// Learned right preconditioner: network kernels (gfx950, BF16 MFMA with FP32 accumulation).
//
//   M(q) = T^{-1} (q + rho * delta(q)),   rho = rms(q)
//
// delta is produced per grid point from four input channels
//   x0 = [ q / rho,  T^{-1}q / rms(T^{-1}q),  D + U,  W + E + S + N ]
// by conv1d over levels (4 -> 32, 5 taps) -> ReLU -> 3x3 horizontal mixing (32 -> 32) -> ReLU
// -> conv1d (32 -> 32, 5 taps) -> ReLU -> conv1d (32 -> 1, 5 taps).  The exact tridiagonal
// solve of the paper's preconditioner (Sec. 2, Eq. 6-7) is kept on both sides; the network
// only adds a correction in residual space, and with its last layer zero M is exactly T^{-1}.
//
// Layouts: activations are [position][32] BF16 (64 bytes per grid point; position = the grid
// index i + nlon (j + nlat k)); x0 is [position][4] BF16.  Each conv layer is a GEMM whose
// K dimension is (tap, input channel): one 16x16x32 MFMA per (tap, 16-wide output tile) over a
// tile of 16 positions.  MFMA operand layout (verified on gfx950): lane l supplies row l % 16
// and K elements 8 (l / 16) .. 8 (l / 16) + 7 of A (and column l % 16 of B); the result lane
// l holds column l % 16 of rows 4 (l / 16) .. 4 (l / 16) + 3.
#include <cmath>

#include "eg_internal.h"

namespace eg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float(static_cast<uint32_t>(u) << 16); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *row)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(row));
}

__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// two floats rounded to BF16 (ties to even) in one 32-bit word, a in the low half
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}

// the network's two vector input channels at one point, BF16: q / rho and z / rho_z (z = T^{-1} q,
// rho, rho_z their root-mean-square values), multiplied in the vectors' precision
template <typename Tv>
__device__ __forceinline__ uint32_t vec_channels(Tv q, Tv z, double inv_rho, double inv_rhoz)
{
    if constexpr (sizeof(Tv) == 4)
        return pack_bf16x2(q * static_cast<float>(inv_rho), z * static_cast<float>(inv_rhoz));
    else
        return pack_bf16x2(static_cast<float>(q * inv_rho), static_cast<float>(z * inv_rhoz));
}

// v if keep, else zero, without a branch (loads stay unconditional, so the compiler can count
// them and wait only for the ones a multiply needs)
__device__ __forceinline__ bf16x8 keep8(bf16x8 v, bool keep)
{
    const uint4 u = __builtin_bit_cast(uint4, v);
    return __builtin_bit_cast(bf16x8, make_uint4(keep ? u.x : 0u, keep ? u.y : 0u, keep ? u.z : 0u, keep ? u.w : 0u));
}

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct Pos {
    int i, j, k;
};

// (i, j, k) of position 0 <= p < n; 32-bit divisions when every position fits in 31 bits (a
// test on a kernel argument, so the branch is uniform)
__device__ __forceinline__ Pos decompose(const NetGeo &g, long p)
{
    Pos r;
    if (g.n <= 0x7fffffffL) {
        const uint32_t u = static_cast<uint32_t>(p), nlon = static_cast<uint32_t>(g.nlon);
        const uint32_t nlat = static_cast<uint32_t>(g.nlat);
        const uint32_t q = u / nlon, k = q / nlat;
        r.i = static_cast<int>(u - q * nlon);
        r.j = static_cast<int>(q - k * nlat);
        r.k = static_cast<int>(k);
    } else {
        r.i = (int)(p % g.nlon);
        const long q = p / g.nlon;
        r.j = (int)(q % g.nlat);
        r.k = (int)(q / g.nlat);
    }
    return r;
}

// neighbour of position p for a vertical tap offset dk (-1 if outside the column)
__device__ __forceinline__ long nb_v(const NetGeo &g, long p, const Pos &x, int dk)
{
    const int k2 = x.k + dk;
    return (k2 < 0 || k2 >= g.nlev) ? -1 : p + (long)dk * g.P;
}

// neighbour for a horizontal offset (di, dj): periodic in longitude, -1 across a pole
__device__ __forceinline__ long nb_h(const NetGeo &g, long p, const Pos &x, int di, int dj)
{
    const int j2 = x.j + dj;
    if (j2 < 0 || j2 >= g.nlat) return -1;
    int i2 = x.i + di;
    if (i2 < 0) i2 += g.nlon;
    else if (i2 >= g.nlon) i2 -= g.nlon;
    return p + (i2 - x.i) + (long)dj * g.nlon;
}

// layer geometry: L1 and L3 are vertical (5 taps, offset t - 2), L2 is horizontal (9 taps)
template <int L> struct LayerGeo {
    static constexpr int T = (L == 2) ? 9 : 5;
    __device__ static __forceinline__ long nb(const NetGeo &g, long p, const Pos &x, int t, bool mirror)
    {
        const int s = mirror ? -1 : 1;
        if constexpr (L == 2) return nb_h(g, p, x, s * (t % 3 - 1), s * (t / 3 - 1));
        else return nb_v(g, p, x, s * (t - 2));
    }
};

__device__ __forceinline__ bool stop_now(const Scalars *sc, int mask)
{
    if (!sc || !mask) return false;
    return ((mask & STOP_DONE) && sc->done) || ((mask & STOP_SKIP) && sc->skip) || ((mask & STOP_HALF) && sc->half);
}

int net_blocks(long n, long per_block, long cap)
{
    long b = (n + per_block - 1) / per_block;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// input channels
// ------------------------------------------------------------------------------------------
template <typename Tv, typename Tc>
__global__ __launch_bounds__(256) void k_net_features(NetGeo g, const Tv *__restrict__ q, const Tv *__restrict__ z0,
                                                      const Tc *__restrict__ a, uint16_t *__restrict__ x0,
                                                      const Scalars *__restrict__ sc, int stop_mask)
{
    if (stop_now(sc, stop_mask)) return;
    const double inv_rho = 1.0 / sqrt(sc->net_q2 / (double)g.n);
    const double inv_rhoz = sc->net_z2 > 0.0 ? 1.0 / sqrt(sc->net_z2 / (double)g.n) : 0.0;
    const long stride = (long)gridDim.x * 256;
    for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < g.n; p += stride) {
        const float c2 = static_cast<float>(a[4 * g.n + p]) + static_cast<float>(a[5 * g.n + p]);
        const float c3 = (static_cast<float>(a[p]) + static_cast<float>(a[g.n + p])) +
                         (static_cast<float>(a[2 * g.n + p]) + static_cast<float>(a[3 * g.n + p]));
        reinterpret_cast<uint2 *>(x0)[p] = make_uint2(vec_channels(q[p], z0[p], inv_rho, inv_rhoz), pack_bf16x2(c2, c3));
    }
}

// ------------------------------------------------------------------------------------------
// Column-marching forward layers.  A wave owns a tile of positions of the level plane (16 for
// the MFMA layers, 64 for the output layer) and walks a chunk of levels upwards, so every
// activation row is read from HBM once per layer: the vertical taps come from a rolling
// register window, the horizontal neighbours of the 3x3 layer from rows the waves of the
// neighbouring tiles read at the same time, and the neighbour offsets in the plane are
// computed once per wave.  Work units (tile, level chunk) are numbered tile-fastest and
// mapped XCD-aware like the SpMV tiles.
// ------------------------------------------------------------------------------------------
struct ColGrid {
    int tiles, kchunk, per_xcd, blocks;
    long units;
};

static ColGrid col_grid(const NetGeo &g, int tile_pos)
{
    ColGrid c;
    c.tiles = (int)((g.P + tile_pos - 1) / tile_pos);
    int chunks = 1;
    while ((long)c.tiles * chunks < 8192 && chunks < g.nlev) chunks *= 2;
    if (chunks > g.nlev) chunks = g.nlev;
    c.kchunk = (g.nlev + chunks - 1) / chunks;
    const int nchunks = (g.nlev + c.kchunk - 1) / c.kchunk;
    c.units = (long)c.tiles * nchunks;
    const long wgs = (c.units + 3) / 4;
    c.per_xcd = (int)((wgs + 7) / 8);
    c.blocks = c.per_xcd * 8;
    return c;
}

__device__ __forceinline__ long col_unit(int per_xcd)
{
    const int b = blockIdx.x;
    return ((long)(b & 7) * per_xcd + (b >> 3)) * 4 + (threadIdx.x >> 6);
}

// Four consecutive output channels of one position (the accumulator started from the bias):
// BF16, then ReLU on the BF16 pairs.  A BF16 number is negative exactly when its 16-bit pattern
// is a negative int16, so a packed int16 max with 0 is the ReLU; rounding is monotone and keeps
// the sign, so this equals rounding max(v, 0) (a negative zero becomes +0).
typedef short s16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v)
{
    const s16x2 r = __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), s16x2{0, 0});
    return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ uint2 relu_pack4(f32x4 acc)
{
    return make_uint2(relu_bf16x2(pack_bf16x2(acc[0], acc[1])), relu_bf16x2(pack_bf16x2(acc[2], acc[3])));
}
__device__ __forceinline__ void store4(uint16_t *dst, f32x4 acc)
{
    *reinterpret_cast<uint2 *>(dst) = relu_pack4(acc);
}
// the bias of output channels 16 nt + 4 grp .. + 3, the accumulator's initial value
__device__ __forceinline__ f32x4 bias4(const float *b, int nt, int grp)
{
    const float *p = b + 16 * nt + 4 * grp;
    return f32x4{p[0], p[1], p[2], p[3]};
}

// ------------------------------------------------------------------------------------------
// conv layer, forward:  out[p][co] = ReLU(bias[co] + sum_{t, ci} W[t][co][ci] in[nb(p, t)][ci])
// The MFMA computes D[co][position] = W[co][K] In[position][K]^T (K = input channels, or
// (tap, channel) for layer 1): lane l ends with output channels 16 nt + 4 (l / 16) .. + 3 of
// position l % 16.  The layer's weights stay in registers for the whole launch.
// ------------------------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(256) void k_conv_fwd(NetGeo g, const uint16_t *__restrict__ in,
                                                  const uint16_t *__restrict__ wf, const float *__restrict__ bias,
                                                  uint16_t *__restrict__ out, const Scalars *__restrict__ sc,
                                                  int stop_mask, int tiles, int kchunk, long units, int per_xcd)
{
    if (stop_now(sc, stop_mask)) return;
    constexpr int T = LayerGeo<L>::T;
    constexpr int NCH = (L == 1) ? 1 : T;   // K chunks of 32
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    // the 3x3 layer keeps its weights (18 KB) in LDS, in each lane's operand order, to leave
    // registers for the next level's loads; the vertical layers keep theirs in registers
    constexpr int NW = (L == 2) ? 18 * 64 : 1;
    __shared__ uint4 wsh[NW];
    if constexpr (L == 2) {
        for (int e = threadIdx.x; e < 18 * 64; e += 256) {
            const int tn = e / 64, l = e % 64;   // tn = 2 t + nt
            wsh[e] = *reinterpret_cast<const uint4 *>(wf + (long)(tn / 2) * 1024 + (16 * (tn % 2) + (l & 15)) * 32 +
                                                      8 * (l >> 4));
        }
        __syncthreads();
    }
    const long unit = col_unit(per_xcd);
    if (unit >= units) return;
    bf16x8 wa[(L == 2) ? 1 : NCH][2];
    if constexpr (L != 2) {
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) wa[c][nt] = ld8(wf + (long)c * 1024 + (16 * nt + m) * 32 + 8 * grp);
    }
    const f32x4 bv0 = bias4(bias, 0, grp), bv1 = bias4(bias, 1, grp);
    const int tile = (int)(unit % tiles);
    const int k0 = (int)(unit / tiles) * kchunk;
    const int k1 = min(g.nlev, k0 + kchunk);
    const long p2 = (long)tile * 16 + m;
    const bool pv = p2 < g.P;
    const long p2s = pv ? p2 : g.P - 1;   // an in-bounds address for the lanes past the plane
    auto emit = [&](int k, f32x4 acc0, f32x4 acc1) {
        if (!pv) return;
        uint16_t *dst = out + ((long)k * g.P + p2) * 32 + 4 * grp;
        store4(dst, acc0);
        store4(dst + 16, acc1);
    };
    if constexpr (L == 2) {
        // the nine horizontal neighbours in the level plane (periodic in longitude, none
        // across a pole), as offsets from p2; bit t of ok marks a neighbour that exists
        const int i = (int)(p2s % g.nlon), j = (int)(p2s / g.nlon);
        int off[9];
        int ok = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int di = t % 3 - 1, dj = t / 3 - 1;
            int i2 = i + di;
            if (i2 < 0) i2 += g.nlon;
            else if (i2 >= g.nlon) i2 -= g.nlon;
            const bool in_plane = j + dj >= 0 && j + dj < g.nlat;
            off[t] = in_plane ? (i2 - i) + dj * g.nlon : 0;   // missing neighbours read p2 itself, masked below
            if (pv && in_plane) ok |= 1 << t;
        }
        // the next level's nine operands are loaded while the current level is multiplied
        auto load9 = [&](int k, bf16x8 *a) {
            const uint16_t *base = in + ((long)k * g.P + p2s) * 32 + 8 * grp;
#pragma unroll
            for (int t = 0; t < 9; ++t) a[t] = ld8(base + (long)off[t] * 32);
        };
        bf16x8 cur[9], nxt[9];
        load9(k0, cur);
        for (int k = k0; k < k1; ++k) {
            // weights are re-read from LDS every level rather than held in 72 registers
            asm volatile("" ::: "memory");
            load9(min(k + 1, k1 - 1), nxt);   // the last level re-reads itself (in bounds, unused)
#pragma unroll
            for (int t = 0; t < 9; ++t) cur[t] = keep8(cur[t], (ok >> t) & 1);
            f32x4 acc0 = bv0, acc1 = bv1;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                acc0 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t) * 64 + lane]), cur[t], acc0);
                acc1 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t + 1) * 64 + lane]), cur[t], acc1);
            }
            emit(k, acc0, acc1);
#pragma unroll
            for (int t = 0; t < 9; ++t) cur[t] = nxt[t];
        }
    } else if constexpr (L == 3) {
        auto row = [&](int kk) -> bf16x8 {
            const int kc = min(max(kk, 0), g.nlev - 1);
            return keep8(ld8(in + ((long)kc * g.P + p2s) * 32 + 8 * grp), pv && kk >= 0 && kk < g.nlev);
        };
        bf16x8 w0 = row(k0 - 2), w1 = row(k0 - 1), w2 = row(k0), w3 = row(k0 + 1), w4 = row(k0 + 2);
        for (int k = k0; k < k1; ++k) {
            const bf16x8 nx = row(k + 3);   // one level ahead
            f32x4 acc0 = bv0, acc1 = bv1;
            acc0 = mfma(wa[0][0], w0, acc0);
            acc1 = mfma(wa[0][1], w0, acc1);
            acc0 = mfma(wa[1][0], w1, acc0);
            acc1 = mfma(wa[1][1], w1, acc1);
            acc0 = mfma(wa[2][0], w2, acc0);
            acc1 = mfma(wa[2][1], w2, acc1);
            acc0 = mfma(wa[3][0], w3, acc0);
            acc1 = mfma(wa[3][1], w3, acc1);
            acc0 = mfma(wa[4][0], w4, acc0);
            acc1 = mfma(wa[4][1], w4, acc1);
            emit(k, acc0, acc1);
            w0 = w1;
            w1 = w2;
            w2 = w3;
            w3 = w4;
            w4 = nx;
        }
    } else {
        // layer 1: K = (tap, channel); lane group grp holds taps 2 grp and 2 grp + 1
        auto row = [&](int kk) -> uint2 {
            const int kc = min(max(kk, 0), g.nlev - 1);
            const uint2 v = reinterpret_cast<const uint2 *>(in)[(long)kc * g.P + p2s];
            const bool keep = pv && kk >= 0 && kk < g.nlev;
            return make_uint2(keep ? v.x : 0u, keep ? v.y : 0u);
        };
        uint2 x0 = row(k0 - 2), x1 = row(k0 - 1), x2 = row(k0), x3 = row(k0 + 1), x4 = row(k0 + 2);
        const uint2 zz = make_uint2(0, 0);
        for (int k = k0; k < k1; ++k) {
            const uint2 nx = row(k + 3);
            const uint2 lo = grp == 0 ? x0 : (grp == 1 ? x2 : (grp == 2 ? x4 : zz));
            const uint2 hi = grp == 0 ? x1 : (grp == 1 ? x3 : zz);
            const bf16x8 a = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
            f32x4 acc0 = bv0, acc1 = bv1;
            acc0 = mfma(wa[0][0], a, acc0);
            acc1 = mfma(wa[0][1], a, acc1);
            emit(k, acc0, acc1);
            x0 = x1;
            x1 = x2;
            x2 = x3;
            x3 = x4;
            x4 = nx;
        }
    }
}

// ------------------------------------------------------------------------------------------
// The 3x3 layer when every tile of 16 positions lies in one latitude row (nlon % 16 == 0): a
// lane loads its own position in the three rows j - 1, j, j + 1, and takes its west and east
// neighbours from the lanes beside it (a DPP shift within the row of 16 lanes that holds one
// channel group); only the tile's two edge columns are loaded separately, as one shared address
// per row.  The taps are multiplied in the order of k_conv_fwd<2>, so the results are the same.
// ------------------------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ bf16x8 dpp8(bf16x8 v)
{
    uint4 u = __builtin_bit_cast(uint4, v);
    u.x = (uint32_t)__builtin_amdgcn_update_dpp((int)u.x, (int)u.x, CTRL, 0xf, 0xf, false);
    u.y = (uint32_t)__builtin_amdgcn_update_dpp((int)u.y, (int)u.y, CTRL, 0xf, 0xf, false);
    u.z = (uint32_t)__builtin_amdgcn_update_dpp((int)u.z, (int)u.z, CTRL, 0xf, 0xf, false);
    u.w = (uint32_t)__builtin_amdgcn_update_dpp((int)u.w, (int)u.w, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(bf16x8, u);
}
constexpr int kDppRowShl1 = 0x101;   // lane m receives lane m + 1 of its row of 16
constexpr int kDppRowShr1 = 0x111;   // lane m receives lane m - 1

__global__ __launch_bounds__(256) void k_conv3x3_rows(NetGeo g, const uint16_t *__restrict__ in,
                                                      const uint16_t *__restrict__ wf, const float *__restrict__ bias,
                                                      uint16_t *__restrict__ out, const Scalars *__restrict__ sc,
                                                      int stop_mask, int tiles, int kchunk, long units, int per_xcd)
{
    if (stop_now(sc, stop_mask)) return;
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    __shared__ uint4 wsh[18 * 64];
    for (int e = threadIdx.x; e < 18 * 64; e += 256) {
        const int tn = e / 64, l = e % 64;   // tn = 2 t + nt
        wsh[e] = *reinterpret_cast<const uint4 *>(wf + (long)(tn / 2) * 1024 + (16 * (tn % 2) + (l & 15)) * 32 +
                                                  8 * (l >> 4));
    }
    __syncthreads();
    const long unit = col_unit(per_xcd);
    if (unit >= units) return;
    const f32x4 bv0 = bias4(bias, 0, grp), bv1 = bias4(bias, 1, grp);
    const int tile = (int)(unit % tiles);
    const int k0 = (int)(unit / tiles) * kchunk;
    const int k1 = min(g.nlev, k0 + kchunk);
    const long t0 = (long)tile * 16, p2 = t0 + m;
    const int nlon = g.nlon;
    const int j = (int)(t0 / nlon), i0 = (int)(t0 % nlon);
    const int il = (i0 == 0) ? nlon - 1 : i0 - 1;        // west of the tile's first column
    const int ir = (i0 + 16 == nlon) ? 0 : i0 + 16;       // east of its last
    const bool rv[3] = {j > 0, true, j < g.nlat - 1};     // rows j - 1, j, j + 1 exist
    long own[3], wl[3], er[3];                             // positions in the level plane
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int jr = rv[r] ? j + r - 1 : j;              // a missing row reads row j, masked below
        own[r] = (long)jr * nlon + (i0 + m);
        wl[r] = (long)jr * nlon + il;
        er[r] = (long)jr * nlon + ir;
    }
    auto load = [&](int k, bf16x8 *a) {
        const uint16_t *base = in + (long)k * g.P * 32 + 8 * grp;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            a[r] = ld8(base + own[r] * 32);
            a[3 + r] = ld8(base + wl[r] * 32);
            a[6 + r] = ld8(base + er[r] * 32);
        }
    };
    bf16x8 cur[9], nxt[9];
    load(k0, cur);
    for (int k = k0; k < k1; ++k) {
        asm volatile("" ::: "memory");
        load(min(k + 1, k1 - 1), nxt);   // the last level re-reads itself (in bounds, unused)
        f32x4 acc0 = bv0, acc1 = bv1;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const bf16x8 o = cur[r];
            bf16x8 w = dpp8<kDppRowShr1>(o);
            bf16x8 e = dpp8<kDppRowShl1>(o);
            w = keep8(m == 0 ? cur[3 + r] : w, rv[r]);
            e = keep8(m == 15 ? cur[6 + r] : e, rv[r]);
            const bf16x8 c = keep8(o, rv[r]);
            const int t = 3 * r;   // taps (di, dj) = (-1, r - 1), (0, r - 1), (1, r - 1)
            acc0 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t) * 64 + lane]), w, acc0);
            acc1 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t + 1) * 64 + lane]), w, acc1);
            acc0 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t + 2) * 64 + lane]), c, acc0);
            acc1 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t + 3) * 64 + lane]), c, acc1);
            acc0 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t + 4) * 64 + lane]), e, acc0);
            acc1 = mfma(__builtin_bit_cast(bf16x8, wsh[(2 * t + 5) * 64 + lane]), e, acc1);
        }
        uint16_t *dst = out + ((long)k * g.P + p2) * 32 + 4 * grp;
        store4(dst, acc0);
        store4(dst + 16, acc1);
#pragma unroll
        for (int t = 0; t < 9; ++t) cur[t] = nxt[t];
    }
}

// The same layer for strips of 64 positions (nlon % 64 == 0): a wave holds four tiles of 16
// consecutive positions, so a tile's first and last lanes take their west / east neighbours
// from the adjacent tile of the same wave (a DPP rotation within the row of 16 lanes); only the
// strip's two edge columns are loaded separately.  Each weight operand is read from LDS once per
// level for the four tiles.  Taps are accumulated in the order of k_conv_fwd<2>.
constexpr int kDppRowRor1 = 0x121;    // lane m receives lane (m - 1) mod 16
constexpr int kDppRowRor15 = 0x12f;   // lane m receives lane (m + 1) mod 16

__global__ __launch_bounds__(256) void k_conv3x3_strip(NetGeo g, const uint16_t *__restrict__ in,
                                                       const uint16_t *__restrict__ wf,
                                                       const float *__restrict__ bias, uint16_t *__restrict__ out,
                                                       const Scalars *__restrict__ sc, int stop_mask, int tiles,
                                                       int kchunk, long units, int per_xcd)
{
    constexpr int NT = 4;   // tiles of 16 positions per wave
    if (stop_now(sc, stop_mask)) return;
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    __shared__ uint4 wsh[18 * 64];
    for (int e = threadIdx.x; e < 18 * 64; e += 256) {
        const int tn = e / 64, l = e % 64;   // tn = 2 t + nt
        wsh[e] = *reinterpret_cast<const uint4 *>(wf + (long)(tn / 2) * 1024 + (16 * (tn % 2) + (l & 15)) * 32 +
                                                  8 * (l >> 4));
    }
    __syncthreads();
    const long unit = col_unit(per_xcd);
    if (unit >= units) return;
    const f32x4 bv0 = bias4(bias, 0, grp), bv1 = bias4(bias, 1, grp);
    const int strip = (int)(unit % tiles);   // `tiles` counts strips of 64 positions here
    const int k0 = (int)(unit / tiles) * kchunk;
    const int k1 = min(g.nlev, k0 + kchunk);
    const int nlon = g.nlon;
    const long t0 = (long)strip * 64;
    const int j = (int)(t0 / nlon), i0 = (int)(t0 % nlon);
    const int il = (i0 == 0) ? nlon - 1 : i0 - 1;          // west of the strip's first column
    const int ir = (i0 + 64 == nlon) ? 0 : i0 + 64;        // east of its last
    const bool rv[3] = {j > 0, true, j < g.nlat - 1};       // rows j - 1, j, j + 1 exist
    int rb[3];                                              // first position of each row used
#pragma unroll
    for (int r = 0; r < 3; ++r) rb[r] = (rv[r] ? j + r - 1 : j) * nlon;   // a missing row reads row j, masked
    // per level: own positions of the four tiles in three rows, then the strip's edges
    auto load = [&](int k, bf16x8 *a) {
        const uint16_t *base = in + (long)k * g.P * 32 + 8 * grp;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int s = 0; s < NT; ++s) a[r * NT + s] = ld8(base + ((long)rb[r] + i0 + 16 * s + m) * 32);
            a[3 * NT + r] = ld8(base + ((long)rb[r] + il) * 32);
            a[3 * NT + 3 + r] = ld8(base + ((long)rb[r] + ir) * 32);
        }
    };
    constexpr int NL = 3 * NT + 6;
    bf16x8 cur[NL], nxt[NL];
    load(k0, cur);
    for (int k = k0; k < k1; ++k) {
        asm volatile("" ::: "memory");
        load(min(k + 1, k1 - 1), nxt);   // the last level re-reads itself (in bounds, unused)
        f32x4 acc[NT][2];
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            acc[s][0] = bv0;
            acc[s][1] = bv1;
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {   // di = c - 1
                const int t = 3 * r + c;
                const bf16x8 w0 = __builtin_bit_cast(bf16x8, wsh[(2 * t) * 64 + lane]);
                const bf16x8 w1 = __builtin_bit_cast(bf16x8, wsh[(2 * t + 1) * 64 + lane]);
#pragma unroll
                for (int s = 0; s < NT; ++s) {
                    bf16x8 v;
                    if (c == 1) {
                        v = cur[r * NT + s];
                    } else if (c == 0) {
                        const bf16x8 in_tile = dpp8<kDppRowShr1>(cur[r * NT + s]);
                        const bf16x8 before = (s > 0) ? dpp8<kDppRowRor1>(cur[r * NT + (s > 0 ? s - 1 : 0)])
                                                      : cur[3 * NT + r];
                        v = (m == 0) ? before : in_tile;
                    } else {
                        const bf16x8 in_tile = dpp8<kDppRowShl1>(cur[r * NT + s]);
                        const bf16x8 after = (s < NT - 1) ? dpp8<kDppRowRor15>(cur[r * NT + (s < NT - 1 ? s + 1 : 0)])
                                                          : cur[3 * NT + 3 + r];
                        v = (m == 15) ? after : in_tile;
                    }
                    v = keep8(v, rv[r]);
                    acc[s][0] = mfma(w0, v, acc[s][0]);
                    acc[s][1] = mfma(w1, v, acc[s][1]);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            uint16_t *dst = out + ((long)k * g.P + t0 + 16 * s + m) * 32 + 4 * grp;
            store4(dst, acc[s][0]);
            store4(dst + 16, acc[s][1]);
        }
#pragma unroll
        for (int t = 0; t < NL; ++t) cur[t] = nxt[t];
    }
}

// ------------------------------------------------------------------------------------------
// conv layer, backward data:  din[p][ci] = [aprev[p][ci] > 0] sum_{t, co} W[t][co][ci] dout[nb(p, -t)][co]
// (the transposed convolution, masked by the derivative of the ReLU that produced aprev)
// ------------------------------------------------------------------------------------------
template <int L>
__global__ __launch_bounds__(256) void k_conv_bwd(NetGeo g, const uint16_t *__restrict__ dout,
                                                  const uint16_t *__restrict__ wt, const uint16_t *__restrict__ aprev,
                                                  uint16_t *__restrict__ din)
{
    constexpr int T = LayerGeo<L>::T;
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    // the weights in MFMA operand order, one 16-byte slot per (tap, output half, lane): held in
    // LDS rather than registers, so more waves fit on a SIMD to hide the loads' latency
    __shared__ uint4 wsh[T * 2 * 64];
    __shared__ __align__(16) uint16_t otile[4][16 * 32];   // per wave: 16 positions x 32 channels
    for (int e = threadIdx.x; e < T * 2 * 64; e += 256) {
        const int t = e >> 7, nt = (e >> 6) & 1, l = e & 63;
        wsh[e] = *reinterpret_cast<const uint4 *>(wt + (long)t * 1024 + (16 * nt + (l & 15)) * 32 + 8 * (l >> 4));
    }
    __syncthreads();
    const long ntiles = (g.n + 15) / 16;
    const long nw = (long)gridDim.x * 4;
    for (long tile = (long)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntiles; tile += nw) {
        const long p = tile * 16 + m;
        const bool pv = p < g.n;
        const long pc = pv ? p : g.n - 1;
        const Pos x = decompose(g, pc);
        // every load is issued before the first multiply (unconditional, at a valid address;
        // a neighbour outside the grid is zeroed afterwards)
        bf16x8 av[T];
        bool ok[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const long q = LayerGeo<L>::nb(g, pc, x, t, true);
            ok[t] = pv && q >= 0;
            av[t] = ld8(dout + (q >= 0 ? q : pc) * 32 + 8 * grp);
        }
        // the tile's result is turned around through LDS so that lane l stores channels
        // 8 (l % 4) .. 8 (l % 4) + 7 of position l / 4 with one 16-byte store; its 8 mask values
        // come with one 16-byte load, issued here with the others
        const long qo = tile * 16 + (lane >> 2);
        const int co = 8 * (lane & 3);
        const uint4 mk = *reinterpret_cast<const uint4 *>(aprev + (qo < g.n ? qo : g.n - 1) * 32 + co);
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        // an opaque copy of the lane index keeps the compiler from hoisting the weight reads
        // out of the loop (which would bring the registers back)
        int wl = lane;
        asm volatile("" : "+v"(wl));
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const bf16x8 a = keep8(av[t], ok[t]);
            acc0 = mfma(a, __builtin_bit_cast(bf16x8, wsh[(2 * t) * 64 + wl]), acc0);
            acc1 = mfma(a, __builtin_bit_cast(bf16x8, wsh[(2 * t + 1) * 64 + wl]), acc1);
        }
        // result lane l: channel m (acc0) and 16 + m (acc1) of positions 4 grp + jj.  The tile
        // is wave-private and LDS serves one wave's accesses in order, so no barrier is needed.
        uint16_t *ot = otile[threadIdx.x >> 6];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            ot[(4 * grp + jj) * 32 + m] = f2bf(acc0[jj]);
            ot[(4 * grp + jj) * 32 + 16 + m] = f2bf(acc1[jj]);
        }
        const uint4 r = *reinterpret_cast<const uint4 *>(ot + (lane >> 2) * 32 + co);
        const uint32_t rv[4] = {r.x, r.y, r.z, r.w}, mv[4] = {mk.x, mk.y, mk.z, mk.w};
        uint32_t ov[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            // f2bf(v * [aprev > 0]): the same bits as masking the FP32 result (a zero keeps v's sign)
            const float lo = bf2f(static_cast<uint16_t>(rv[h] & 0xffffu)), hi = bf2f(static_cast<uint16_t>(rv[h] >> 16));
            const float mlo = bf2f(static_cast<uint16_t>(mv[h] & 0xffffu)) > 0.f ? 1.f : 0.f;
            const float mhi = bf2f(static_cast<uint16_t>(mv[h] >> 16)) > 0.f ? 1.f : 0.f;
            ov[h] = static_cast<uint32_t>(f2bf(lo * mlo)) | (static_cast<uint32_t>(f2bf(hi * mhi)) << 16);
        }
        if (qo < g.n) *reinterpret_cast<uint4 *>(din + qo * 32 + co) = make_uint4(ov[0], ov[1], ov[2], ov[3]);
    }
}


// ------------------------------------------------------------------------------------------
// Backward data of the vertical 32 -> 32 layer (layer 3) as a column march, the structure of
// the forward kernel: each dout row is loaded once and the five taps come from a rolling
// window of levels.  The MFMA forms D[ci][position] = Wt[t][ci][co] dout[position][co]^T
// (Wt the transposed weights [tap][ci][co]); tap t pairs with level k + 2 - t, and the taps
// are accumulated in the order t = 0 .. 4.  Lane l ends with input channels 16 nt + 4 (l / 16)
// .. + 3 of position l % 16, masked by [aprev > 0] (8-byte loads and stores).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv_bwd_col(NetGeo g, const uint16_t *__restrict__ dout,
                                                      const uint16_t *__restrict__ wt,
                                                      const uint16_t *__restrict__ aprev, uint16_t *__restrict__ din,
                                                      int tiles, int kchunk, long units, int per_xcd)
{
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    const long unit = col_unit(per_xcd);
    if (unit >= units) return;
    bf16x8 wa[5][2];
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) wa[t][nt] = ld8(wt + (long)t * 1024 + (16 * nt + m) * 32 + 8 * grp);
    const int tile = (int)(unit % tiles);
    const int k0 = (int)(unit / tiles) * kchunk;
    const int k1 = min(g.nlev, k0 + kchunk);
    const long p2 = (long)tile * 16 + m;
    const bool pv = p2 < g.P;
    const long p2s = pv ? p2 : g.P - 1;   // an in-bounds address for the lanes past the plane
    auto row = [&](int kk) -> bf16x8 {
        const int kc = min(max(kk, 0), g.nlev - 1);
        return keep8(ld8(dout + ((long)kc * g.P + p2s) * 32 + 8 * grp), pv && kk >= 0 && kk < g.nlev);
    };
    // f2bf(v * [a > 0]) for four channels: v FP32 results, a the BF16 activations
    auto masked = [](f32x4 v, uint2 a) -> uint2 {
        const float m0 = bf2f(static_cast<uint16_t>(a.x & 0xffffu)) > 0.f ? 1.f : 0.f;
        const float m1 = bf2f(static_cast<uint16_t>(a.x >> 16)) > 0.f ? 1.f : 0.f;
        const float m2 = bf2f(static_cast<uint16_t>(a.y & 0xffffu)) > 0.f ? 1.f : 0.f;
        const float m3 = bf2f(static_cast<uint16_t>(a.y >> 16)) > 0.f ? 1.f : 0.f;
        return make_uint2(static_cast<uint32_t>(f2bf(v[0] * m0)) | (static_cast<uint32_t>(f2bf(v[1] * m1)) << 16),
                          static_cast<uint32_t>(f2bf(v[2] * m2)) | (static_cast<uint32_t>(f2bf(v[3] * m3)) << 16));
    };
    bf16x8 w0 = row(k0 - 2), w1 = row(k0 - 1), w2 = row(k0), w3 = row(k0 + 1), w4 = row(k0 + 2);
    for (int k = k0; k < k1; ++k) {
        const bf16x8 nx = row(k + 3);   // one level ahead
        const long ob = ((long)k * g.P + p2s) * 32 + 4 * grp;
        const uint2 a0 = *reinterpret_cast<const uint2 *>(aprev + ob);
        const uint2 a1 = *reinterpret_cast<const uint2 *>(aprev + ob + 16);
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        acc0 = mfma(wa[0][0], w4, acc0);
        acc1 = mfma(wa[0][1], w4, acc1);
        acc0 = mfma(wa[1][0], w3, acc0);
        acc1 = mfma(wa[1][1], w3, acc1);
        acc0 = mfma(wa[2][0], w2, acc0);
        acc1 = mfma(wa[2][1], w2, acc1);
        acc0 = mfma(wa[3][0], w1, acc0);
        acc1 = mfma(wa[3][1], w1, acc1);
        acc0 = mfma(wa[4][0], w0, acc0);
        acc1 = mfma(wa[4][1], w0, acc1);
        if (pv) {
            *reinterpret_cast<uint2 *>(din + ob) = masked(acc0, a0);
            *reinterpret_cast<uint2 *>(din + ob + 16) = masked(acc1, a1);
        }
        w0 = w1;
        w1 = w2;
        w2 = w3;
        w3 = w4;
        w4 = nx;
    }
}
// ------------------------------------------------------------------------------------------
// Weight gradient of the 32 -> 32 layers through LDS (layers 2 and 3):
//   dW[t][co][ci] = sum_p dout[p][co] in[nb(p, t)][ci],   db[co] = sum_p dout[p][co]
// One workgroup (one partial row) walks chunks of 32 consecutive positions.  A chunk needs
// T + 1 tiles of 32 positions x 32 channels: dout, and the input at each tap's neighbours.
// Wave w loads tiles w, w + 4, w + 8 with 16-byte loads, a lane taking 8 channels of two
// adjacent positions, and writes them to LDS transposed ([channel][position]) as packed
// position pairs, so each MFMA operand (8 consecutive positions of one channel) is a single
// 16-byte LDS read; K = 32 positions per MFMA.  Wave w multiplies taps w, w + 4, w + 8 (its
// accumulators: 16 floats per tap).  Two chunks are in flight in registers: the loads of
// chunk c + 2 (in grid-stride steps) are issued before the multiplications of chunk c, so
// their latency is hidden behind two chunks of work, and each chunk costs two barriers.
// ------------------------------------------------------------------------------------------
template <int NTPW> struct DwBuf {
    uint4 v[NTPW][2];   // [tile of this wave][even, odd position]
    bool ok[NTPW][2];   // false: the value is outside the grid and counts as zero
};

// wave wv's tiles of chunk ch.  The loads are unconditional (an address outside the grid is
// replaced by the position itself and flagged), so the compiler can count them and a put
// waits only for its own chunk.
template <int L, int NTPW>
__device__ __forceinline__ DwBuf<NTPW> dw_fetch(const NetGeo g, const uint16_t *dout, const uint16_t *in, long ch,
                                                int wv, int pp, int cq)
{
    constexpr int NT = LayerGeo<L>::T + 1;
    DwBuf<NTPW> r;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const long p = ch * 32 + 2 * pp + e;
        const bool pv = p < g.n;
        const long pc = pv ? p : g.n - 1;
        const Pos x = decompose(g, pc);
#pragma unroll
        for (int a = 0; a < NTPW; ++a) {
            const int tile = wv + 4 * a < NT ? wv + 4 * a : 0;
            const long q = (tile == 0) ? pc : LayerGeo<L>::nb(g, pc, x, tile - 1, false);
            r.ok[a][e] = pv && q >= 0;
            r.v[a][e] = *reinterpret_cast<const uint4 *>(((tile == 0) ? dout : in) + (q >= 0 ? q : pc) * 32 + 8 * cq);
        }
    }
    return r;
}

template <int L>
__global__ __launch_bounds__(256) void k_conv_dw_lds(NetGeo g, const uint16_t *__restrict__ dout,
                                                     const uint16_t *__restrict__ in, float *__restrict__ part,
                                                     int add)
{
    static_assert(L == 2 || L == 3, "32 -> 32 layers only");
    constexpr int T = LayerGeo<L>::T;
    constexpr int NT = T + 1;           // tile 0: dout; tile 1 + t: input at tap t
    constexpr int TPW = (NT + 3) / 4;   // tiles loaded per wave
    constexpr int TW = (T + 3) / 4;     // taps multiplied per wave
    constexpr int PITCH = 40;           // bf16 per LDS row (80 bytes: 16-byte aligned rows)
    __shared__ __align__(16) uint16_t tl[NT][32 * PITCH];
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int pp = lane >> 2, cq = lane & 3;   // loader lane: positions 2 pp, 2 pp + 1; channels 8 cq .. 8 cq + 7
    f32x4 acc[TW][2][2];
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) acc[a][b][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) bsum[c] = 0.f;
    const long nchunks = (g.n + 31) / 32;
    const long G = gridDim.x;

    auto fetch = [&](long ch) { return dw_fetch<L, TPW>(g, dout, in, ch, wv, pp, cq); };
    // channel c = 8 cq + h of the two positions as one dword: (even | odd << 16)
    auto put = [&](const DwBuf<TPW> &r) {
#pragma unroll
        for (int a = 0; a < TPW; ++a) {
            const int tile = wv + 4 * a;
            if (tile >= NT) break;
            const uint32_t ke = r.ok[a][0] ? 0xffffffffu : 0u, ko = r.ok[a][1] ? 0xffffffffu : 0u;
            const uint32_t ev[4] = {r.v[a][0].x & ke, r.v[a][0].y & ke, r.v[a][0].z & ke, r.v[a][0].w & ke};
            const uint32_t od[4] = {r.v[a][1].x & ko, r.v[a][1].y & ko, r.v[a][1].z & ko, r.v[a][1].w & ko};
            uint32_t *dst = reinterpret_cast<uint32_t *>(tl[tile]);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                dst[((8 * cq + 2 * h) * PITCH + 2 * pp) / 2] = (ev[h] & 0xffffu) | (od[h] << 16);
                dst[((8 * cq + 2 * h + 1) * PITCH + 2 * pp) / 2] = (ev[h] >> 16) | (od[h] & 0xffff0000u);
            }
            if (tile == 0) {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    bsum[2 * h] += bf2f(static_cast<uint16_t>(ev[h] & 0xffffu)) + bf2f(static_cast<uint16_t>(od[h] & 0xffffu));
                    bsum[2 * h + 1] += bf2f(static_cast<uint16_t>(ev[h] >> 16)) + bf2f(static_cast<uint16_t>(od[h] >> 16));
                }
            }
        }
    };
    auto multiply = [&]() {
        bf16x8 A[2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
            A[mt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(tl[0] + (16 * mt + m) * PITCH + 8 * grp));
#pragma unroll
        for (int a = 0; a < TW; ++a) {
            const int t = wv + 4 * a;
            if (t >= T) break;
            bf16x8 B[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                B[nt] = __builtin_bit_cast(bf16x8,
                                           *reinterpret_cast<const uint4 *>(tl[1 + t] + (16 * nt + m) * PITCH + 8 * grp));
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) acc[a][mt][nt] = mfma(A[mt], B[nt], acc[a][mt][nt]);
        }
    };

    // chunks ch (from b0) and ch + G (from b1) per trip; every wave meets every barrier.  A
    // fetch past the last chunk re-reads the last one (valid addresses, never used; operator
    // grids have n >= 3, so there is a last chunk).
    const long last = nchunks - 1;
    long ch = blockIdx.x;
    DwBuf<TPW> b0 = fetch(ch < last ? ch : last);
    DwBuf<TPW> b1 = fetch(ch + G < last ? ch + G : last);
    for (; ch < nchunks; ch += 2 * G) {
        __syncthreads();   // the previous chunk's tiles are no longer read
        put(b0);
        b0 = fetch(ch + 2 * G < last ? ch + 2 * G : last);
        __syncthreads();
        multiply();
        if (ch + G >= nchunks) break;
        __syncthreads();
        put(b1);
        b1 = fetch(ch + 3 * G < last ? ch + 3 * G : last);
        __syncthreads();
        multiply();
    }

    float *dst = part + (long)blockIdx.x * kNetParams;
    const int off = (L == 2) ? kNetOffW2 : kNetOffW3;
    // result lane l: co = 16 mt + 4 grp + jj, ci = 16 nt + m.  The previous values are read
    // unconditionally (all of them before the first add) and used only when adding.
#pragma unroll
    for (int a = 0; a < TW; ++a) {
        const int t = wv + 4 * a;
        if (t >= T) break;
        float prev[2][2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    prev[mt][nt][jj] = dst[off + t * 1024 + (16 * mt + 4 * grp + jj) * 32 + 16 * nt + m];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                    dst[off + t * 1024 + (16 * mt + 4 * grp + jj) * 32 + 16 * nt + m] =
                        add ? prev[mt][nt][jj] + acc[a][mt][nt][jj] : acc[a][mt][nt][jj];
    }
    if (wv == 0) {
        // bias: lanes with the same cq hold the same channels for different positions
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float v = bsum[c];
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lane < 4) {
                float &o = dst[((L == 2) ? kNetOffB2 : kNetOffB3) + 8 * cq + c];
                o = add ? o + v : v;
            }
        }
    }
}

constexpr int kLevelBatch = 8;   // levels whose loads a column march issues together

// ------------------------------------------------------------------------------------------
// Weight gradients of the two layers with few weights, as column marches on the vector ALU.
// A workgroup is 8 streams of 32 lanes (lane = channel); a stream takes whole columns of the
// level plane and walks their levels, so every activation row is read once (64 contiguous
// bytes per stream) and the few values of the other factor come from a rolling window of
// five levels (a broadcast load per level).  The 8 streams' sums are added in a fixed order in
// LDS and written as the workgroup's partial row.
//   output layer: dW4[t][c] = sum_p drho(p) a3[p + (t-2) P][c], db4 = sum_p drho(p), drho = rho u
//   layer 1:      dW1[t][co][ci] = sum_p dh1[p][co] x0[p + (t-2) P][ci], db1[co] = sum_p dh1[p][co]
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_net_out_dw_col(NetGeo g, const float *__restrict__ u,
                                                        const uint16_t *__restrict__ a3, float *__restrict__ part,
                                                        const Scalars *__restrict__ sc, int add)
{
    const float rho = static_cast<float>(sqrt(sc->net_q2 / (double)g.n));
    const int c = threadIdx.x & 31, st = threadIdx.x >> 5;
    const long nst = (long)gridDim.x * 8;
    float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    // loads at a clamped level, zeroed outside the column afterwards (no branch around a load)
    auto dr = [&](long col, int k) -> float {
        const int kc = k < 0 ? 0 : (k < g.nlev ? k : g.nlev - 1);
        const float v = rho * u[col + (long)kc * g.P];
        return (k >= 0 && k < g.nlev) ? v : 0.f;
    };
    for (long col = (long)blockIdx.x * 8 + st; col < g.P; col += nst) {
        // d[t] = drho at level kk + 2 - t
        float d0 = dr(col, 2), d1 = dr(col, 1), d2 = dr(col, 0), d3 = 0.f, d4 = 0.f;
        // levels in batches, each batch's loads issued together; past the top the
        // activation and drho are zero, so the extra steps add exact zeros
        for (int k0 = 0; k0 < g.nlev; k0 += kLevelBatch) {
            uint16_t araw[kLevelBatch];
            float uraw[kLevelBatch];
#pragma unroll
            for (int j = 0; j < kLevelBatch; ++j) {   // raw loads only: scaling and masking come at use
                const int kk = k0 + j;
                const int kc = kk < g.nlev ? kk : g.nlev - 1;
                const int ku = kk + 3 < g.nlev ? kk + 3 : g.nlev - 1;
                araw[j] = a3[(col + (long)kc * g.P) * 32 + c];
                uraw[j] = u[col + (long)ku * g.P];
            }
#pragma unroll
            for (int j = 0; j < kLevelBatch; ++j) {
                const float a = (k0 + j < g.nlev) ? bf2f(araw[j]) : 0.f;
                acc[0] += d0 * a;
                acc[1] += d1 * a;
                acc[2] += d2 * a;
                acc[3] += d3 * a;
                acc[4] += d4 * a;
                bacc += d2;
                d4 = d3;
                d3 = d2;
                d2 = d1;
                d1 = d0;
                d0 = (k0 + j + 3 < g.nlev) ? rho * uraw[j] : 0.f;
            }
        }
    }
    __shared__ float red[8][161];
#pragma unroll
    for (int t = 0; t < 5; ++t) red[st][t * 32 + c] = acc[t];
    if (c == 0) red[st][160] = bacc;
    __syncthreads();
    if (threadIdx.x <= 160) {
        float v = 0.f;
        for (int r = 0; r < 8; ++r) v += red[r][threadIdx.x];
        float *dst = part + (long)blockIdx.x * kNetParams;
        float &o = (threadIdx.x < 160) ? dst[kNetOffW4 + threadIdx.x] : dst[kNetOffB4];
        o = add ? o + v : v;
    }
}

__global__ __launch_bounds__(256) void k_conv_dw1_col(NetGeo g, const uint16_t *__restrict__ dout,
                                                      const uint16_t *__restrict__ x0, float *__restrict__ part,
                                                      int add)
{
    const int co = threadIdx.x & 31, st = threadIdx.x >> 5;
    const long nst = (long)gridDim.x * 8;
    float acc[5][4];
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) acc[t][ci] = 0.f;
    float bacc = 0.f;
    // loads at a clamped level, zeroed outside the column afterwards (no branch around a load)
    auto xin = [&](long col, int k) -> uint2 {
        const int kc = k < 0 ? 0 : (k < g.nlev ? k : g.nlev - 1);
        const uint2 v = reinterpret_cast<const uint2 *>(x0)[col + (long)kc * g.P];
        const bool in = k >= 0 && k < g.nlev;
        return make_uint2(in ? v.x : 0u, in ? v.y : 0u);
    };
    auto ch = [](uint2 v, int ci) -> float {
        const uint32_t w = (ci < 2) ? v.x : v.y;
        return bf2f(static_cast<uint16_t>((ci & 1) ? (w >> 16) : (w & 0xffffu)));
    };
    for (long col = (long)blockIdx.x * 8 + st; col < g.P; col += nst) {
        // w[t] = x0 at level k + t - 2
        uint2 w0 = xin(col, -2), w1 = xin(col, -1), w2 = xin(col, 0), w3 = xin(col, 1), w4 = xin(col, 2);
        // levels in batches, each batch's loads issued together; past the top dout and x0
        // are zero, so the extra steps add exact zeros
        for (int k0 = 0; k0 < g.nlev; k0 += kLevelBatch) {
            uint16_t draw[kLevelBatch];
            uint2 nx[kLevelBatch];
#pragma unroll
            for (int j = 0; j < kLevelBatch; ++j) {   // raw loads only: masking comes at use
                const int k = k0 + j;
                const int kc = k < g.nlev ? k : g.nlev - 1;
                const int kx = k + 3 < g.nlev ? k + 3 : g.nlev - 1;
                draw[j] = dout[(col + (long)kc * g.P) * 32 + co];
                nx[j] = reinterpret_cast<const uint2 *>(x0)[col + (long)kx * g.P];
            }
#pragma unroll
            for (int j = 0; j < kLevelBatch; ++j) {
                const float dv = (k0 + j < g.nlev) ? bf2f(draw[j]) : 0.f;
                bacc += dv;
#pragma unroll
                for (int ci = 0; ci < 4; ++ci) {
                    acc[0][ci] += dv * ch(w0, ci);
                    acc[1][ci] += dv * ch(w1, ci);
                    acc[2][ci] += dv * ch(w2, ci);
                    acc[3][ci] += dv * ch(w3, ci);
                    acc[4][ci] += dv * ch(w4, ci);
                }
                w0 = w1;
                w1 = w2;
                w2 = w3;
                w3 = w4;
                const bool top = k0 + j + 3 < g.nlev;
                w4 = make_uint2(top ? nx[j].x : 0u, top ? nx[j].y : 0u);
            }
        }
    }
    __shared__ float red[8][5 * 128 + 32];
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int ci = 0; ci < 4; ++ci) red[st][t * 128 + co * 4 + ci] = acc[t][ci];
    red[st][640 + co] = bacc;
    __syncthreads();
    float *dst = part + (long)blockIdx.x * kNetParams;
    for (int e = threadIdx.x; e < 672; e += 256) {
        float v = 0.f;
        for (int r = 0; r < 8; ++r) v += red[r][e];
        float &o = (e < 640) ? dst[kNetOffW1 + e] : dst[kNetOffB1 + (e - 640)];
        o = add ? o + v : v;
    }
}

// ------------------------------------------------------------------------------------------
// output layer (32 -> 1, 5 vertical taps) fused with  q' = q + rho * delta
// One lane per position of the level plane, marching up a chunk of levels: each input row
// a3[kk] is read once and its five tap sums s_t = sum_c W4[t][c] a3[kk][c] are added to the
// pending outputs of levels kk + 2 - t; level kk - 2 is complete after input kk.
// ------------------------------------------------------------------------------------------
template <typename Tv>
__global__ __launch_bounds__(256) void k_net_out(NetGeo g, const uint16_t *__restrict__ a3,
                                                 const float *__restrict__ w4, const float *__restrict__ theta,
                                                 const Tv *__restrict__ q, Tv *__restrict__ qout,
                                                 float *__restrict__ delta, const Scalars *__restrict__ sc,
                                                 int stop_mask, int tiles, int kchunk, long units, int per_xcd)
{
    if (stop_now(sc, stop_mask)) return;
    __shared__ float w[160];
    if (threadIdx.x < 160) w[threadIdx.x] = w4[threadIdx.x];
    __syncthreads();
    const long unit = col_unit(per_xcd);
    if (unit >= units) return;
    const float b4 = theta[kNetOffB4];
    const double rho = sqrt(sc->net_q2 / (double)g.n);
    const int tile = (int)(unit % tiles);
    const int k0 = (int)(unit / tiles) * kchunk;
    const int k1 = min(g.nlev, k0 + kchunk);
    const long p2 = (long)tile * 64 + (threadIdx.x & 63);
    if (p2 >= g.P) return;
    // r[d] accumulates the output of level kk - 2 + d
    float r[5] = {b4, b4, b4, b4, b4};
    // input rows are loaded one level ahead (clamped to the grid; a clamped row is not used)
    auto ldrow = [&](int kk, uint4 *u) {
        const int kc = min(max(kk, 0), g.nlev - 1);
        const uint4 *row = reinterpret_cast<const uint4 *>(a3 + ((long)kc * g.P + p2) * 32);
#pragma unroll
        for (int v = 0; v < 4; ++v) u[v] = row[v];
    };
    uint4 cur[4], nxt[4];
    ldrow(k0 - 2, cur);
    for (int kk = k0 - 2; kk < k1 + 2; ++kk) {
        // keeps the weights in LDS (read as broadcasts every level) instead of 160 registers
        asm volatile("" ::: "memory");
        ldrow(kk + 1, nxt);
        if (kk >= 0 && kk < g.nlev) {
            float s[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint4 u = cur[v];
                const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int c = 8 * v + 2 * h;
                    const float lo = __uint_as_float(wd[h] << 16), hi = __uint_as_float(wd[h] & 0xffff0000u);
#pragma unroll
                    for (int t = 0; t < 5; ++t) s[t] += w[t * 32 + c] * lo + w[t * 32 + c + 1] * hi;
                }
            }
#pragma unroll
            for (int d = 0; d < 5; ++d) r[d] += s[4 - d];
        }
        const int k = kk - 2;
        if (k >= k0 && k < k1) {
            const long p = (long)k * g.P + p2;
            if (delta) delta[p] = r[0];
            qout[p] = static_cast<Tv>(static_cast<double>(q[p]) + rho * static_cast<double>(r[0]));
        }
        r[0] = r[1];
        r[1] = r[2];
        r[2] = r[3];
        r[3] = r[4];
        r[4] = b4;
#pragma unroll
        for (int v = 0; v < 4; ++v) cur[v] = nxt[v];
    }
}

// ------------------------------------------------------------------------------------------
// Inference: layer 3 (conv1d 32 -> 32, 5 taps) and the output layer (conv1d 32 -> 1, 5 taps)
// in one column march, so the layer-3 activations never go to HBM.  Per level kk the MFMA
// forms the 16 positions' a3(kk) (bias, ReLU and BF16 rounding as the two-kernel path stores
// them), a second MFMA the five tap sums of each position, and the sums join the pending
// outputs of levels kk + 2 - t as in k_net_out.  Output level k needs a3 at k - 2 .. k + 2,
// which needs a2 at k - 4 .. k + 4: a level chunk recomputes the a3 levels it shares with its
// neighbours.
// ------------------------------------------------------------------------------------------
template <typename Tv>
__global__ __launch_bounds__(256) void k_conv3_out(NetGeo g, const uint16_t *__restrict__ a2,
                                                   const uint16_t *__restrict__ w3f, const float *__restrict__ w4,
                                                   const float *__restrict__ theta, const Tv *__restrict__ q,
                                                   Tv *__restrict__ qout, float *__restrict__ delta,
                                                   const Scalars *__restrict__ sc, int stop_mask, int tiles,
                                                   int kchunk, long units, int per_xcd)
{
    if (stop_now(sc, stop_mask)) return;
    const long unit = col_unit(per_xcd);
    if (unit >= units) return;
    const int lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    bf16x8 wa[5][2];
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) wa[c][nt] = ld8(w3f + (long)c * 1024 + (16 * nt + m) * 32 + 8 * grp);
    // this lane's channels 16 nt + 4 grp + jj: layer-3 bias
    const f32x4 bv0 = bias4(theta + kNetOffB3, 0, grp), bv1 = bias4(theta + kNetOffB3, 1, grp);
    // The output layer is one more MFMA per level, D[t][position] = W4[t][K] a3[position][K]:
    // with the K index 8 grp + 4 nt + jj standing for channel 16 nt + 4 grp + jj, the B operand
    // is this lane's own eight a3 values, and A is row t = m of W4 (taps 0..4; rows 5..15 zero)
    // in the same channel order.  W4 is held BF16-exact, so the products are exact.
    uint32_t wd[4];
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        const int c = 16 * (i / 4) + 4 * grp + (i % 4);   // channel of K element 8 grp + i
        const uint32_t lo = m < 5 ? f2bf(w4[m * 32 + c]) : 0u, hi = m < 5 ? f2bf(w4[m * 32 + c + 1]) : 0u;
        wd[i / 2] = lo | (hi << 16);
    }
    const bf16x8 w4a = __builtin_bit_cast(bf16x8, make_uint4(wd[0], wd[1], wd[2], wd[3]));
    const float b4 = theta[kNetOffB4];
    const double rho = sqrt(sc->net_q2 / (double)g.n);
    const int tile = (int)(unit % tiles);
    const int k0 = (int)(unit / tiles) * kchunk;
    const int k1 = min(g.nlev, k0 + kchunk);
    const long p2 = (long)tile * 16 + m;
    const bool pv = p2 < g.P;
    const long p2s = pv ? p2 : g.P - 1;   // an in-bounds address for the lanes past the plane
    auto row = [&](int kk) -> bf16x8 {
        const int kc = min(max(kk, 0), g.nlev - 1);
        return keep8(ld8(a2 + ((long)kc * g.P + p2s) * 32 + 8 * grp), pv && kk >= 0 && kk < g.nlev);
    };
    // a2 window of the first a3 level computed (it moves one level per computed a3 level) and
    // the next two rows in flight
    const int ka = max(k0 - 2, 0);
    bf16x8 v0 = row(ka - 2), v1 = row(ka - 1), v2 = row(ka), v3 = row(ka + 1), v4 = row(ka + 2);
    bf16x8 n0 = row(ka + 3), n1 = row(ka + 4);
    // r[d] accumulates the output of level kk - 2 + d
    float r[5] = {b4, b4, b4, b4, b4};
    for (int kk = k0 - 2; kk < k1 + 2; ++kk) {
        if (kk >= 0 && kk < g.nlev) {
            const bf16x8 nx = row(kk + 5);   // three levels ahead
            f32x4 acc[2] = {bv0, bv1};
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                acc[nt] = mfma(wa[0][nt], v0, acc[nt]);
                acc[nt] = mfma(wa[1][nt], v1, acc[nt]);
                acc[nt] = mfma(wa[2][nt], v2, acc[nt]);
                acc[nt] = mfma(wa[3][nt], v3, acc[nt]);
                acc[nt] = mfma(wa[4][nt], v4, acc[nt]);
            }
            // a3 as the two-kernel path stores it (BF16, ReLU), packed in K order
            const uint2 a0 = relu_pack4(acc[0]), a1 = relu_pack4(acc[1]);
            const f32x4 so = mfma(w4a, __builtin_bit_cast(bf16x8, make_uint4(a0.x, a0.y, a1.x, a1.y)),
                                  f32x4{0.f, 0.f, 0.f, 0.f});
            // lane (m, 0) holds the tap sums t = 0..3 of position m, lane (m, 1) holds t = 4
            const float s4 = __shfl_down(so[0], 16);
            const float st[5] = {so[0], so[1], so[2], so[3], s4};
#pragma unroll
            for (int d = 0; d < 5; ++d) r[d] += st[4 - d];
            v0 = v1;
            v1 = v2;
            v2 = v3;
            v3 = v4;
            v4 = n0;
            n0 = n1;
            n1 = nx;
        }
        const int k = kk - 2;
        if (k >= k0 && k < k1 && grp == 0 && pv) {
            const long p = (long)k * g.P + p2;
            if (delta) delta[p] = r[0];
            qout[p] = static_cast<Tv>(static_cast<double>(q[p]) + rho * static_cast<double>(r[0]));
        }
        r[0] = r[1];
        r[1] = r[2];
        r[2] = r[3];
        r[3] = r[4];
        r[4] = b4;
    }
}

// ------------------------------------------------------------------------------------------
// The operator's static input channels (D + U, W + E + S + N as BF16, one 32-bit word per
// grid point), formed as k_net_features forms them; the FP32 coefficients are the FP32
// roundings of the FP64 ones, so one array serves both precisions.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_net_static(long n, const double *__restrict__ a, uint32_t *__restrict__ fs)
{
    const long stride = (long)gridDim.x * 256;
    for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) {
        const float c2 = static_cast<float>(a[4 * n + p]) + static_cast<float>(a[5 * n + p]);
        const float c3 = (static_cast<float>(a[p]) + static_cast<float>(a[n + p])) +
                         (static_cast<float>(a[2 * n + p]) + static_cast<float>(a[3 * n + p]));
        fs[p] = pack_bf16x2(c2, c3);
    }
}

// ------------------------------------------------------------------------------------------
// The whole inference in one launch (nlon a multiple of 64): input channels, layer 1, the 3x3
// layer, layer 3 and the output layer, with a1 and a2 handed on in LDS and registers instead
// of HBM.  A workgroup of eight waves (two per SIMD) owns 4 latitude rows x 64 longitudes and
// marches up the levels; wave w owns tiles 2 (w % 2) and 2 (w % 2) + 1 of 16 positions in row
// w / 2.  Step s does
//   * layer 1 at level s on the block's rows, the row on each side, and one more tile holding
//     the west and east halo columns of those six rows (25 tiles, spread over the waves).  Its
//     input channels are formed on the fly from q, T^{-1} q and the static channels as
//     k_net_features forms them, in a window of five levels per tile (the loads of level
//     s + 3 are issued at the start of the step and consumed at its end); the result goes to
//     an LDS plane [row][8-channel block][column], double-buffered by level, zero on rows
//     outside the grid (the poles);
//   * a workgroup barrier;
//   * a2 of level s - 1 (written by this wave at step s - 1) read back from a wave-private LDS
//     tile in the operand layout of layer 3 (channels 8 grp .. 8 grp + 7 of its position),
//     joining a window of five levels; the 3x3 layer at level s for the wave's two tiles,
//     operands from the LDS plane, weights from LDS, the result written to the other half of
//     the wave's LDS tile (read back after the next barrier);
//   * layer 3 at level s - 3 from the window and its output-layer tap sums (as k_conv3_out),
//     and the output of level s - 5:  q' = q + rho delta.
// Every product and sum is taken in the order of the layered kernels (k_net_features,
// k_conv_fwd<1>, k_conv3x3_strip, k_conv3_out), so the result is bitwise theirs.  Offsets are
// 32-bit byte offsets from the arrays' bases (the launcher checks n * sizeof(Tv) < 2^32).
// ------------------------------------------------------------------------------------------
constexpr int kFuRows = 4;                // latitude rows per workgroup
constexpr int kFuCols = 64;               // longitudes per workgroup
constexpr int kFuWaves = 8;               // two per row, two per SIMD
constexpr int kFuA1Rows = kFuRows + 2;    // layer-1 rows: the block's and one on each side
constexpr int kFuA1Cols = kFuCols + 2;    // with the west and east halo columns
constexpr int kFuA1Elems = kFuA1Rows * 4 * kFuA1Cols;   // 16-byte elements of one plane
constexpr int kFuL1Tiles = 4 * kFuA1Rows + 1;
constexpr int kFuL1PerWave = (kFuL1Tiles + kFuWaves - 1) / kFuWaves;

template <typename T> __device__ __forceinline__ T ld_off(const T *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}
template <typename T> __device__ __forceinline__ void st_off(T *base, uint32_t off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off) = v;
}

// a wave-uniform double held in scalar registers
__device__ __forceinline__ double uniform_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

template <typename Tv>
__global__ __launch_bounds__(64 * kFuWaves) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_net_fused(
    NetGeo g, const Tv *__restrict__ q, const Tv *__restrict__ z0, const uint32_t *__restrict__ fstat,
    const uint16_t *__restrict__ w1f, const uint16_t *__restrict__ w2f, const uint16_t *__restrict__ w3f,
    const float *__restrict__ w4, const float *__restrict__ theta, Tv *__restrict__ qout, float *__restrict__ delta,
    const Scalars *__restrict__ sc, int stop_mask, int nstrips, int nblocks, int per_xcd)
{
    if (stop_now(sc, stop_mask)) return;
    const int blk = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);   // XCD-aware, as the SpMV tiles
    if (blk >= nblocks) return;                                        // whole workgroup
    __shared__ uint4 w2s[18 * 64];                     // 3x3 weights in each lane's operand order
    __shared__ uint4 a1s[2][kFuA1Elems];               // layer-1 plane, [row][block][column]
    __shared__ uint4 a2s[2][kFuWaves][2 * 4 * 16];     // per wave: [tile][block][position]
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, m = lane & 15, grp = lane >> 4;
    const int nlon = g.nlon, nlat = g.nlat, nlev = g.nlev;
    const long P = g.P;
    const int j0 = (blk / nstrips) * kFuRows, i0 = (blk % nstrips) * kFuCols;
    for (int e = threadIdx.x; e < 18 * 64; e += 64 * kFuWaves) {
        const int tn = e / 64, l = e % 64;   // tn = 2 t + nt
        w2s[e] = *reinterpret_cast<const uint4 *>(w2f + (long)(tn / 2) * 1024 + (16 * (tn % 2) + (l & 15)) * 32 +
                                                  8 * (l >> 4));
    }

    bf16x8 w1a[2], w3a[5][2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) w1a[nt] = ld8(w1f + (16 * nt + m) * 32 + 8 * grp);
#pragma unroll
    for (int c = 0; c < 5; ++c)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) w3a[c][nt] = ld8(w3f + (long)c * 1024 + (16 * nt + m) * 32 + 8 * grp);
    // biases of layers 1-3 as accumulator initial values, [layer][nt][grp], read from LDS at
    // each use (registers are the scarce resource here)
    __shared__ f32x4 bias_s[3][2][4];
    if (threadIdx.x < 24) {
        const int ly = threadIdx.x / 8, nt = (threadIdx.x / 4) % 2, gq = threadIdx.x % 4;
        bias_s[ly][nt][gq] = bias4(theta + (ly == 0 ? kNetOffB1 : (ly == 1 ? kNetOffB2 : kNetOffB3)), nt, gq);
    }
    // both layer-1 planes start at zero: rows outside the grid (the poles) are never written
    for (int e = threadIdx.x; e < 2 * kFuA1Elems; e += 64 * kFuWaves) (&a1s[0][0])[e] = make_uint4(0, 0, 0, 0);
    __syncthreads();   // the 3x3 weights, the biases and the zeroed planes, before layer 1
    uint32_t wd[4];
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
        const int c = 16 * (i / 4) + 4 * grp + (i % 4);
        const uint32_t lo = m < 5 ? f2bf(w4[m * 32 + c]) : 0u, hi = m < 5 ? f2bf(w4[m * 32 + c + 1]) : 0u;
        wd[i / 2] = lo | (hi << 16);
    }
    const bf16x8 w4a = __builtin_bit_cast(bf16x8, make_uint4(wd[0], wd[1], wd[2], wd[3]));
    const float b4 = theta[kNetOffB4];
    const double inv_rho = uniform_f64(1.0 / sqrt(sc->net_q2 / (double)g.n));
    const double inv_rhoz = uniform_f64(sc->net_z2 > 0.0 ? 1.0 / sqrt(sc->net_z2 / (double)g.n) : 0.0);
    const double rho = uniform_f64(sqrt(sc->net_q2 / (double)g.n));
    // lane group grp supplies layer 1's taps 2 grp and 2 grp + 1: masks that pick them from the
    // window without indexing it by grp (an indexed window would be placed in scratch memory)
    const uint32_t g0 = grp == 0 ? ~0u : 0u, g1 = grp == 1 ? ~0u : 0u, g2 = grp == 2 ? ~0u : 0u;
    const uint32_t step_v = static_cast<uint32_t>(P * (long)sizeof(Tv)), step_f = static_cast<uint32_t>(P * 4);

    // layer-1 tiles of this wave: u = wv + 8 t.  Tile u < 24 is row u / 4 of the layer-1 rows
    // (grid row j0 - 1 + u / 4), columns 16 (u % 4) + m of the block; tile 24 holds the west
    // (lanes 0..5) and east (lanes 6..11) halo columns of the six rows, lanes 12..15 unused.
    uint32_t pos1[kFuL1PerWave];   // plane position (in bounds)
    int dst1[kFuL1PerWave];        // LDS element (8-byte units) of this lane's channel group, -1: none
    bool val1[kFuL1PerWave];       // the position lies inside the grid
#pragma unroll
    for (int t = 0; t < kFuL1PerWave; ++t) {
        const int u = wv + kFuWaves * t;
        int rr = -1, col = 0, i = i0;
        if (u < 4 * kFuA1Rows) {
            rr = u >> 2;
            col = 1 + 16 * (u & 3) + m;
            i = i0 + 16 * (u & 3) + m;
        } else if (u == 4 * kFuA1Rows && m < 2 * kFuA1Rows) {
            const bool east = m >= kFuA1Rows;
            rr = east ? m - kFuA1Rows : m;
            col = east ? kFuA1Cols - 1 : 0;
            i = east ? (i0 + kFuCols == nlon ? 0 : i0 + kFuCols) : (i0 == 0 ? nlon - 1 : i0 - 1);
        }
        const int j = j0 - 1 + rr;
        val1[t] = rr >= 0 && j >= 0 && j < nlat;
        pos1[t] = val1[t] ? static_cast<uint32_t>(j * nlon + i) : 0u;
        dst1[t] = rr < 0 ? -1 : ((rr * 4 + (grp >> 1)) * kFuA1Cols + col) * 2 + (grp & 1);
    }
    struct Raw {
        Tv q, z;
        uint32_t f;
    };
    auto load_raw = [&](int t, int L) -> Raw {
        const uint32_t lc = static_cast<uint32_t>(min(max(L, 0), nlev - 1));
        return Raw{ld_off(q, pos1[t] * (uint32_t)sizeof(Tv) + lc * step_v),
                   ld_off(z0, pos1[t] * (uint32_t)sizeof(Tv) + lc * step_v), ld_off(fstat, pos1[t] * 4u + lc * step_f)};
    };
    // input channels at level L (zero outside the column; positions outside the grid compute
    // values that are never stored)
    auto channels = [&](int L, const Raw &v) -> uint2 {
        const bool keep = L >= 0 && L < nlev;   // uniform
        return keep ? make_uint2(vec_channels(v.q, v.z, inv_rho, inv_rhoz), v.f) : make_uint2(0u, 0u);
    };
    // Rolling windows are rings indexed by level mod 5 (the loop below is unrolled by five, so
    // every index is a constant and nothing is copied from slot to slot):
    //   xw   input channels of levels st - 1 .. st + 3 (layer 1 runs one level ahead),
    //   vw   a2 of levels st - 5 .. st - 1,
    //   racc pending outputs of levels st - 5 .. st - 1 (started from the output bias).
    uint2 xw[kFuL1PerWave][5];
    Raw nxt[kFuL1PerWave];       // level st + 4, in flight during step st
    // layer 1 at level L from the window (taps 2 grp, 2 grp + 1 are levels L - 2 + 2 grp,
    // L - 1 + 2 grp, in slots (L - 2 + tap) mod 5), into LDS plane L & 1
    uint2 *a1w = reinterpret_cast<uint2 *>(&a1s[0][0]);
    auto layer1 = [&](auto l_c, int L) {
        constexpr int LM = decltype(l_c)::value;   // L mod 5
        uint2 *pl = a1w + (L & 1) * (kFuA1Elems * 2);
#pragma unroll
        for (int t = 0; t < kFuL1PerWave; ++t) {
            if (wv + kFuWaves * t >= kFuL1Tiles) continue;   // wave-uniform
            const uint2 x0 = xw[t][(LM + 3) % 5], x1 = xw[t][(LM + 4) % 5], x2 = xw[t][LM % 5],
                        x3 = xw[t][(LM + 1) % 5], x4 = xw[t][(LM + 2) % 5];
            const uint2 lo = make_uint2((x0.x & g0) | (x2.x & g1) | (x4.x & g2), (x0.y & g0) | (x2.y & g1) | (x4.y & g2));
            const uint2 hi = make_uint2((x1.x & g0) | (x3.x & g1), (x1.y & g0) | (x3.y & g1));
            const bf16x8 a = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
            const f32x4 acc0 = mfma(w1a[0], a, bias_s[0][0][grp]);
            const f32x4 acc1 = mfma(w1a[1], a, bias_s[0][1][grp]);
            if (val1[t]) {
                pl[dst1[t]] = relu_pack4(acc0);                        // channels 4 grp .. + 3
                pl[dst1[t] + 2 * 2 * kFuA1Cols] = relu_pack4(acc1);    // channels 16 + 4 grp .. + 3
            }
        }
    };
#pragma unroll
    for (int t = 0; t < kFuL1PerWave; ++t)
        if (wv + kFuWaves * t < kFuL1Tiles)
#pragma unroll
            for (int L = -2; L <= 2; ++L) xw[t][(L + 5) % 5] = channels(L, load_raw(t, L));
    layer1(std::integral_constant<int, 0>{}, 0);
#pragma unroll
    for (int t = 0; t < kFuL1PerWave; ++t)   // level 3 replaces level -2
        if (wv + kFuWaves * t < kFuL1Tiles) xw[t][3] = channels(3, load_raw(t, 3));
    __syncthreads();   // layer 1 of level 0

    // this wave's output row and the positions of its two tiles
    const int lr = wv >> 1, hc = kFuCols / 2 * (wv & 1);
    const int jo = j0 + lr;
    const bool row_ok = jo < nlat;
    const uint32_t po = static_cast<uint32_t>((row_ok ? jo : 0) * nlon + i0 + hc + m);   // + 16 s for tile s
    bf16x8 vw[2][5];
    float racc[2][5];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            vw[s][d] = zero8();
            racc[s][d] = b4;
        }

    // one step; PH = st mod 5
    auto step = [&](auto ph_c, int st) {
        constexpr int PH = decltype(ph_c)::value;
        const int buf = st & 1;
        const int k = st - 5;   // output level of this step
        // loads consumed at the end of the step: layer-1 inputs of level st + 4, q of level k
        if (st + 1 < nlev) {
#pragma unroll
            for (int t = 0; t < kFuL1PerWave; ++t)
                if (wv + kFuWaves * t < kFuL1Tiles) nxt[t] = load_raw(t, st + 4);
        }
        const uint32_t ko = static_cast<uint32_t>(min(max(k, 0), nlev - 1));
        Tv qo[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) qo[s] = ld_off(q, (po + 16 * s) * (uint32_t)sizeof(Tv) + ko * step_v);
        // ---- layer 1 at level st + 1, into the plane the 3x3 layer reads next step ----
        if (st + 1 < nlev) layer1(std::integral_constant<int, (PH + 1) % 5>{}, st + 1);
        // ---- a2 of level st - 1 joins the window ----
        if (st >= 1 && st - 1 < nlev) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
                vw[s][(PH + 4) % 5] = __builtin_bit_cast(bf16x8, a2s[buf ^ 1][wv][(s * 4 + grp) * 16 + m]);
        } else {
#pragma unroll
            for (int s = 0; s < 2; ++s) vw[s][(PH + 4) % 5] = zero8();
        }
        // ---- the 3x3 layer at level st for this wave's two tiles ----
        auto conv3 = [&]() {
            if (st >= nlev) return;
            const uint4 *pl = &a1s[buf][0];
            const f32x4 b20 = bias_s[1][0][grp], b21 = bias_s[1][1][grp];
            f32x4 acc[2][2] = {{b20, b21}, {b20, b21}};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {   // tap t = 3 r + c: (di, dj) = (c - 1, r - 1)
                    const int t = 3 * r + c;
                    const bf16x8 wa0 = __builtin_bit_cast(bf16x8, w2s[(2 * t) * 64 + lane]);
                    const bf16x8 wa1 = __builtin_bit_cast(bf16x8, w2s[(2 * t + 1) * 64 + lane]);
                    const uint4 *rowp = pl + ((lr + r) * 4 + grp) * kFuA1Cols + hc + c + m;   // column 1 + hc + m + c - 1
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const bf16x8 v = __builtin_bit_cast(bf16x8, rowp[16 * s]);
                        acc[s][0] = mfma(wa0, v, acc[s][0]);
                        acc[s][1] = mfma(wa1, v, acc[s][1]);
                    }
                }
            }
            uint2 *tw = reinterpret_cast<uint2 *>(&a2s[buf][wv][0]);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    tw[((s * 4 + 2 * nt + (grp >> 1)) * 16 + m) * 2 + (grp & 1)] = relu_pack4(acc[s][nt]);
        };
        // ---- layer 3 at level kk = st - 3 (a2 of levels st - 5 .. st - 1), output of level k ----
        auto layer3 = [&]() {
            const int kk = st - 3;
            if (kk < 0 || kk >= nlev) return;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                f32x4 acc[2] = {bias_s[2][0][grp], bias_s[2][1][grp]};
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                    for (int c = 0; c < 5; ++c) acc[nt] = mfma(w3a[c][nt], vw[s][(PH + c) % 5], acc[nt]);
                const uint2 a0 = relu_pack4(acc[0]), a1 = relu_pack4(acc[1]);
                const f32x4 so = mfma(w4a, __builtin_bit_cast(bf16x8, make_uint4(a0.x, a0.y, a1.x, a1.y)),
                                      f32x4{0.f, 0.f, 0.f, 0.f});
                const float s4 = __shfl_down(so[0], 16);
                const float stp[5] = {so[0], so[1], so[2], so[3], s4};
                // output level st - 5 + d (slot (PH + d) % 5) takes tap 4 - d of this a3 level
#pragma unroll
                for (int d = 0; d < 5; ++d) racc[s][(PH + d) % 5] += stp[4 - d];
            }
        };
        // the two are independent within a step; the two waves of a SIMD (w and w + 4) take
        // them in opposite order, so one streams LDS operands while the other multiplies
        // register operands
        if (wv < 4) {
            conv3();
            layer3();
        } else {
            layer3();
            conv3();
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (k >= 0 && k < nlev && grp == 0 && row_ok) {
                const uint32_t e = po + 16 * s + static_cast<uint32_t>(k) * static_cast<uint32_t>(P);   // element
                if (delta) st_off(delta, e * 4u, racc[s][PH]);
                st_off(qout, e * (uint32_t)sizeof(Tv),
                       static_cast<Tv>(static_cast<double>(qo[s]) + rho * static_cast<double>(racc[s][PH])));
            }
            racc[s][PH] = b4;   // the slot's next level is st
        }
        // level st + 4 enters the layer-1 window (in the slot of level st - 1)
        if (st + 1 < nlev) {
#pragma unroll
            for (int t = 0; t < kFuL1PerWave; ++t)
                if (wv + kFuWaves * t < kFuL1Tiles) xw[t][(PH + 4) % 5] = channels(st + 4, nxt[t]);
        }
        // layer 1 of level st + 1 and the a2 tile of level st are complete; the plane and the
        // tile read this step may be written again
        __syncthreads();
    };
    if constexpr (sizeof(Tv) == 4) {
        // nlev + 5 steps, padded to a multiple of five with steps that do nothing but the barrier
        const int nsteps = (nlev + 5 + 4) / 5 * 5;
        for (int st = 0; st < nsteps; st += 5) {
            step(std::integral_constant<int, 0>{}, st);
            step(std::integral_constant<int, 1>{}, st + 1);
            step(std::integral_constant<int, 2>{}, st + 2);
            step(std::integral_constant<int, 3>{}, st + 3);
            step(std::integral_constant<int, 4>{}, st + 4);
        }
    } else {
        // FP64 vectors: unrolled by five the kernel would not fit two waves per SIMD; every
        // step takes phase 0 and the rings are turned by one slot after it
        for (int st = 0; st < nlev + 5; ++st) {
            step(std::integral_constant<int, 0>{}, st);
#pragma unroll
            for (int t = 0; t < kFuL1PerWave; ++t) {
                const uint2 x = xw[t][0];
#pragma unroll
                for (int d = 0; d < 4; ++d) xw[t][d] = xw[t][d + 1];
                xw[t][4] = x;
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const bf16x8 v = vw[s][0];
                const float r = racc[s][0];
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    vw[s][d] = vw[s][d + 1];
                    racc[s][d] = racc[s][d + 1];
                }
                vw[s][4] = v;
                racc[s][4] = r;
            }
        }
    }
}

// Backward of the output layer:  dδ = rho u;  dh3[p][c] = [a3 > 0] sum_t W4[t][c] dδ[p - (t - 2) P]
__global__ __launch_bounds__(256) void k_net_out_bwd(NetGeo g, const float *__restrict__ u,
                                                     const uint16_t *__restrict__ a3, const float *__restrict__ w4,
                                                     uint16_t *__restrict__ dh3, const Scalars *__restrict__ sc)
{
    __shared__ float w[160];
    if (threadIdx.x < 160) w[threadIdx.x] = w4[threadIdx.x];
    __syncthreads();
    const float rho = static_cast<float>(sqrt(sc->net_q2 / (double)g.n));
    const long stride = (long)gridDim.x * 256;
    for (long p = (long)blockIdx.x * 256 + threadIdx.x; p < g.n; p += stride) {
        const Pos x = decompose(g, p);
        // the five loads at valid addresses first (a level outside the column reads p and is
        // zeroed afterwards), so they are in flight together
        float ur[5];
        bool in[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) {
            const long nb = nb_v(g, p, x, -(t - 2));
            in[t] = nb >= 0;
            ur[t] = u[nb >= 0 ? nb : p];
        }
        float dd[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) dd[t] = in[t] ? rho * ur[t] : 0.f;
        const uint4 *row = reinterpret_cast<const uint4 *>(a3 + p * 32);
        uint4 *orow = reinterpret_cast<uint4 *>(dh3 + p * 32);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint4 ain = row[v];
            const uint32_t wd[4] = {ain.x, ain.y, ain.z, ain.w};
            uint32_t od[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                float o[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int c = 8 * v + 2 * h + e;
                    float s = 0.f;
#pragma unroll
                    for (int t = 0; t < 5; ++t) s += w[t * 32 + c] * dd[t];
                    const float av = e ? __uint_as_float(wd[h] & 0xffff0000u) : __uint_as_float(wd[h] << 16);
                    o[e] = av > 0.f ? s : 0.f;
                }
                od[h] = static_cast<uint32_t>(f2bf(o[0])) | (static_cast<uint32_t>(f2bf(o[1])) << 16);
            }
            orow[v] = make_uint4(od[0], od[1], od[2], od[3]);
        }
    }
}


// ------------------------------------------------------------------------------------------
// loss pieces:  g = 2 (m - e) / ||e||^2
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_net_gseed(long n, const float *__restrict__ m, const float *__restrict__ e,
                                                   float *__restrict__ gout, const Scalars *__restrict__ sc)
{
    const float s = static_cast<float>(2.0 / sc->net_ee);
    const long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) gout[i] = s * (m[i] - e[i]);
}

// diff = m - e (for the loss numerator)
__global__ __launch_bounds__(256) void k_net_diff(long n, const float *__restrict__ m, const float *__restrict__ e,
                                                  float *__restrict__ out)
{
    const long stride = (long)gridDim.x * 256;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) out[i] = m[i] - e[i];
}

// ------------------------------------------------------------------------------------------
// z = T^{-T} y per column from the LU factors (l, inv, c) of T = L U:
//   U^T u = y :  ~u_k = y_k + c_{k-1} ~u_{k-1},  u_k = inv_k ~u_k
//   L^T z = u :  z_k = u_k + l_{k+1} z_{k+1}
// One lane per column.  The columns are few next to the lanes of the chip (one per horizontal
// point), so the level walks load eight levels at a time (at clamped levels, all issued
// before the first use) to keep more loads in flight than the recurrence alone would.
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_thomas_t(TriView<float> tv, const float *__restrict__ y,
                                                  float *__restrict__ z)
{
    constexpr int B = 8;
    const long col = (long)blockIdx.x * 256 + threadIdx.x;
    if (col >= tv.P) return;
    const long P = tv.P, n = tv.n;
    const int nlev = tv.nlev;
    const float *lf = tv.f, *invf = tv.f + n, *cf = tv.f + 2 * n;
    float ut = 0.f, cprev = 0.f;
    for (int k0 = 0; k0 < nlev; k0 += B) {
        float yv[B], iv[B], cv[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const long c = col + (long)(k0 + j < nlev ? k0 + j : nlev - 1) * P;
            yv[j] = y[c];
            iv[j] = invf[c];
            cv[j] = cf[c];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (k0 + j < nlev) {
                ut = yv[j] + cprev * ut;
                z[col + (long)(k0 + j) * P] = iv[j] * ut;
                cprev = cv[j];
            }
        }
    }
    float zz = 0.f, lnext = 0.f;
    for (int k1 = nlev - 1; k1 >= 0; k1 -= B) {
        float zv[B], lv[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const long c = col + (long)(k1 - j >= 0 ? k1 - j : 0) * P;
            zv[j] = z[c];
            lv[j] = lf[c];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (k1 - j >= 0) {
                zz = zv[j] + lnext * zz;
                z[col + (long)(k1 - j) * P] = zz;
                lnext = lv[j];
            }
        }
    }
}

// ------------------------------------------------------------------------------------------
// y = A^T x in FP32 (gradient of the residual-space loss):
//   (A^T x)_c = C_c x_c - W(c+1) x(c+1) - E(c-1) x(c-1) - S(j+1) x(j+1) - N(j-1) x(j-1)
//               - D(k+1) x(k+1) - U(k-1) x(k-1),   C = m + sum of the six couplings
// (longitude periodic; terms across a pole, the bottom or the top are absent)
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_spmv_t(NetGeo g, const float *__restrict__ a, const float *__restrict__ mg,
                                                const float *__restrict__ x, float *__restrict__ y)
{
    const long n = g.n;
    const long stride = (long)gridDim.x * 256;
    for (long c = (long)blockIdx.x * 256 + threadIdx.x; c < n; c += stride) {
        const Pos p = decompose(g, c);
        const long cw = c - p.i + (p.i == 0 ? g.nlon - 1 : p.i - 1);
        const long ce = c - p.i + (p.i == g.nlon - 1 ? 0 : p.i + 1);
        float diag = mg[c];
#pragma unroll
        for (int d = 0; d < 6; ++d) diag += a[d * n + c];
        // the four conditional neighbours load at a valid index (c itself when absent) and are
        // zeroed afterwards, so no load waits behind a branch
        const bool hn = p.j < g.nlat - 1, hs = p.j > 0, hu = p.k < g.nlev - 1, hd = p.k > 0;
        const long cn = hn ? c + g.nlon : c, cs = hs ? c - g.nlon : c;
        const long cu = hu ? c + g.P : c, cd = hd ? c - g.P : c;
        const float tn = a[2 * n + cn] * x[cn], ts = a[3 * n + cs] * x[cs];
        const float tu = a[4 * n + cu] * x[cu], td = a[5 * n + cd] * x[cd];
        float s = diag * x[c];
        s -= a[ce] * x[ce];              // row c+1 couples to c through its W coupling
        s -= a[n + cw] * x[cw];          // row c-1 through its E coupling
        if (hn) s -= tn;
        if (hs) s -= ts;
        if (hu) s -= tu;
        if (hd) s -= td;
        y[c] = s;
    }
}

void launch_spmv_t(const NetGeo &g, const float *a, const float *m, const float *x, float *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_spmv_t, dim3(net_blocks(g.n, 1024, 8192)), dim3(256), 0, s, g, a, m, x, y);
}

// ------------------------------------------------------------------------------------------
// parameters: gradient reduction, Adam, BF16 copies
// ------------------------------------------------------------------------------------------
// grad[i] = scale * sum over the partial rows of part[row][i]: eight interleaved running sums
// (rows r = 8 q + c go to sum c) combined in a fixed tree, so the result is deterministic.
__global__ __launch_bounds__(256) void k_net_reduce(const float *__restrict__ part, int rows, float scale,
                                                    float *__restrict__ grad)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kNetParams) return;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int r = 0;
    for (; r + 8 <= rows; r += 8)
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] += part[(long)(r + c) * kNetParams + i];
    for (; r < rows; ++r) s[0] += part[(long)r * kNetParams + i];
    grad[i] = scale * (((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
}

__device__ void refresh_one(const NetDev &d, int i, float v)
{
    const uint16_t b = f2bf(v);
    if (i < kNetOffB1) {                    // W1[t][co][ci] -> w1f[co][t*4 + ci]
        const int t = i / 128, co = (i % 128) / 4, ci = i % 4;
        d.w1f[co * 32 + t * 4 + ci] = b;
    } else if (i >= kNetOffW2 && i < kNetOffB2) {
        const int r = i - kNetOffW2, t = r / 1024, co = (r % 1024) / 32, ci = r % 32;
        d.w2f[t * 1024 + co * 32 + ci] = b;
        d.w2b[t * 1024 + ci * 32 + co] = b;
    } else if (i >= kNetOffW3 && i < kNetOffB3) {
        const int r = i - kNetOffW3, t = r / 1024, co = (r % 1024) / 32, ci = r % 32;
        d.w3f[t * 1024 + co * 32 + ci] = b;
        d.w3b[t * 1024 + ci * 32 + co] = b;
    } else if (i >= kNetOffW4 && i < kNetOffB4) {
        d.w4[i - kNetOffW4] = bf2f(b);
    }
}

__global__ __launch_bounds__(256) void k_net_refresh(NetDev d)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < kNetParams) refresh_one(d, i, d.theta[i]);
}

__global__ __launch_bounds__(256) void k_net_adam(NetDev d, float lr, float b1, float b2, float eps, float c1,
                                                  float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= kNetParams) return;
    const float gr = d.grad[i];
    const float m = b1 * d.adam_m[i] + (1.f - b1) * gr;
    const float v = b2 * d.adam_v[i] + (1.f - b2) * gr * gr;
    d.adam_m[i] = m;
    d.adam_v[i] = v;
    const float th = d.theta[i] - lr * (m * c1) / (sqrtf(v * c2) + eps);
    d.theta[i] = th;
    refresh_one(d, i, th);
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
template <typename Tv, typename Tc>
void launch_net_features(const NetGeo &g, const Tv *q, const Tv *z0, const Tc *a, uint16_t *x0, const Scalars *sc,
                         int stop_mask, hipStream_t s)
{
    hipLaunchKernelGGL((k_net_features<Tv, Tc>), dim3(net_blocks(g.n, 1024, 8192)), dim3(256), 0, s, g, q, z0, a, x0,
                       sc, stop_mask);
}

// layers 1 and 2 (x0 -> a1 -> a2)
static void launch_net_layers12(const NetGeo &g, const NetDev &d, const NetActs &act, const Scalars *sc, int stop_mask,
                                hipStream_t s)
{
    const ColGrid c = col_grid(g, 16);
    hipLaunchKernelGGL((k_conv_fwd<1>), dim3(c.blocks), dim3(256), 0, s, g, act.x0, d.w1f, d.theta + kNetOffB1, act.a1,
                       sc, stop_mask, c.tiles, c.kchunk, c.units, c.per_xcd);
    if (g.nlon % 64 == 0) {
        const ColGrid c4 = col_grid(g, 64);
        hipLaunchKernelGGL(k_conv3x3_strip, dim3(c4.blocks), dim3(256), 0, s, g, act.a1, d.w2f, d.theta + kNetOffB2,
                           act.a2, sc, stop_mask, c4.tiles, c4.kchunk, c4.units, c4.per_xcd);
    } else if (g.nlon % 16 == 0)
        hipLaunchKernelGGL(k_conv3x3_rows, dim3(c.blocks), dim3(256), 0, s, g, act.a1, d.w2f, d.theta + kNetOffB2,
                           act.a2, sc, stop_mask, c.tiles, c.kchunk, c.units, c.per_xcd);
    else
        hipLaunchKernelGGL((k_conv_fwd<2>), dim3(c.blocks), dim3(256), 0, s, g, act.a1, d.w2f, d.theta + kNetOffB2,
                           act.a2, sc, stop_mask, c.tiles, c.kchunk, c.units, c.per_xcd);
}

void launch_net_forward_layers(const NetGeo &g, const NetDev &d, const NetActs &act, const Scalars *sc, int stop_mask,
                               hipStream_t s)
{
    launch_net_layers12(g, d, act, sc, stop_mask, s);
    const ColGrid c = col_grid(g, 16);
    hipLaunchKernelGGL((k_conv_fwd<3>), dim3(c.blocks), dim3(256), 0, s, g, act.a2, d.w3f, d.theta + kNetOffB3, act.a3,
                       sc, stop_mask, c.tiles, c.kchunk, c.units, c.per_xcd);
}

template <typename Tv>
void launch_net_forward_fused(const NetGeo &g, const NetDev &d, const NetActs &act, const Tv *q, Tv *qout,
                              float *delta, const Scalars *sc, int stop_mask, hipStream_t s)
{
    launch_net_layers12(g, d, act, sc, stop_mask, s);
    const ColGrid c = col_grid(g, 16);
    hipLaunchKernelGGL((k_conv3_out<Tv>), dim3(c.blocks), dim3(256), 0, s, g, act.a2, d.w3f, d.w4, d.theta, q, qout,
                       delta, sc, stop_mask, c.tiles, c.kchunk, c.units, c.per_xcd);
}

template <typename Tv>
void launch_net_out(const NetGeo &g, const NetDev &d, const NetActs &act, const Tv *q, Tv *qout, float *delta,
                    const Scalars *sc, int stop_mask, hipStream_t s)
{
    const ColGrid c = col_grid(g, 64);
    hipLaunchKernelGGL((k_net_out<Tv>), dim3(c.blocks), dim3(256), 0, s, g, act.a3, d.w4, d.theta, q, qout, delta, sc,
                       stop_mask, c.tiles, c.kchunk, c.units, c.per_xcd);
}

// the one-launch inference takes blocks of 64 longitudes and 32-bit byte offsets (FP64 vectors)
bool net_fused_ok(const NetGeo &g) { return g.nlon % kFuCols == 0 && (unsigned long)g.n * 8 < (1ul << 32); }

void launch_net_static(long n, const double *a64, uint32_t *fs, hipStream_t s)
{
    hipLaunchKernelGGL(k_net_static, dim3(net_blocks(n, 1024, 8192)), dim3(256), 0, s, n, a64, fs);
}

template <typename Tv>
void launch_net_infer(const NetGeo &g, const NetDev &d, const Tv *q, const Tv *z0, const uint32_t *fstat, Tv *qout,
                      float *delta, const Scalars *sc, int stop_mask, hipStream_t s)
{
    const int nstrips = g.nlon / kFuCols;
    const long nb = (long)nstrips * ((g.nlat + kFuRows - 1) / kFuRows);
    const int per_xcd = (int)((nb + 7) / 8);
    hipLaunchKernelGGL((k_net_fused<Tv>), dim3(per_xcd * 8), dim3(64 * kFuWaves), 0, s, g, q, z0, fstat, d.w1f, d.w2f, d.w3f,
                       d.w4, d.theta, qout, delta, sc, stop_mask, nstrips, (int)nb, per_xcd);
}

void launch_thomas_t(const TriView<float> &tv, const float *y, float *z, hipStream_t s)
{
    hipLaunchKernelGGL(k_thomas_t, dim3((unsigned)((tv.P + 255) / 256)), dim3(256), 0, s, tv, y, z);
}

void launch_net_gseed(long n, const float *m, const float *e, float *g, const Scalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_net_gseed, dim3(net_blocks(n, 1024, 8192)), dim3(256), 0, s, n, m, e, g, sc);
}

void launch_net_diff(long n, const float *m, const float *e, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_net_diff, dim3(net_blocks(n, 1024, 8192)), dim3(256), 0, s, n, m, e, out);
}

// Backward through the network for one pair: per-row partial weight gradients are written
// (first pair of a batch) or added (later pairs) into d.part; launch_net_grad then sums the
// rows once per batch.
void launch_net_backward(const NetGeo &g, const NetDev &d, const NetActs &act, const float *u, const Scalars *sc,
                         int first, hipStream_t s)
{
    const int rows = kNetPartRows;
    const int add = first ? 0 : 1;
    // output layer
    hipLaunchKernelGGL(k_net_out_bwd, dim3(net_blocks(g.n, 1024, 8192)), dim3(256), 0, s, g, u, act.a3, d.w4, act.d1,
                       sc);
    hipLaunchKernelGGL(k_net_out_dw_col, dim3(rows), dim3(256), 0, s, g, u, act.a3, d.part, sc, add);
    const int nb = net_blocks((g.n + 15) / 16, 4 * 8, 4096);
    // layer 3: dW3 from (dh3, a2); dh2 = bwd(dh3) masked by a2
    hipLaunchKernelGGL((k_conv_dw_lds<3>), dim3(rows), dim3(256), 0, s, g, act.d1, act.a2, d.part, add);
    const ColGrid c = col_grid(g, 16);
    hipLaunchKernelGGL(k_conv_bwd_col, dim3(c.blocks), dim3(256), 0, s, g, act.d1, d.w3b, act.a2, act.d2, c.tiles,
                       c.kchunk, c.units, c.per_xcd);
    // layer 2: dW2 from (dh2, a1); dh1 = bwd(dh2) masked by a1
    hipLaunchKernelGGL((k_conv_dw_lds<2>), dim3(rows), dim3(256), 0, s, g, act.d2, act.a1, d.part, add);
    hipLaunchKernelGGL((k_conv_bwd<2>), dim3(nb), dim3(256), 0, s, g, act.d2, d.w2b, act.a1, act.d1);
    // layer 1: dW1 from (dh1, x0)
    hipLaunchKernelGGL(k_conv_dw1_col, dim3(rows), dim3(256), 0, s, g, act.d1, act.x0, d.part, add);
}

void launch_net_grad(const NetDev &d, float scale, hipStream_t s)
{
    hipLaunchKernelGGL(k_net_reduce, dim3((kNetParams + 255) / 256), dim3(256), 0, s, d.part, kNetPartRows, scale,
                       d.grad);
}

void launch_net_refresh(const NetDev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_net_refresh, dim3((kNetParams + 255) / 256), dim3(256), 0, s, d);
}

void launch_net_adam(const NetDev &d, float lr, int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f / (1.f - powf(b1, (float)step));
    const float c2 = 1.f / (1.f - powf(b2, (float)step));
    hipLaunchKernelGGL(k_net_adam, dim3((kNetParams + 255) / 256), dim3(256), 0, s, d, lr, b1, b2, eps, c1, c2);
}

template void launch_net_features<double, double>(const NetGeo &, const double *, const double *, const double *,
                                                  uint16_t *, const Scalars *, int, hipStream_t);
template void launch_net_features<float, double>(const NetGeo &, const float *, const float *, const double *,
                                                 uint16_t *, const Scalars *, int, hipStream_t);
template void launch_net_features<float, float>(const NetGeo &, const float *, const float *, const float *,
                                                uint16_t *, const Scalars *, int, hipStream_t);
template void launch_net_forward_fused<double>(const NetGeo &, const NetDev &, const NetActs &, const double *,
                                               double *, float *, const Scalars *, int, hipStream_t);
template void launch_net_forward_fused<float>(const NetGeo &, const NetDev &, const NetActs &, const float *, float *,
                                              float *, const Scalars *, int, hipStream_t);
template void launch_net_infer<double>(const NetGeo &, const NetDev &, const double *, const double *,
                                       const uint32_t *, double *, float *, const Scalars *, int, hipStream_t);
template void launch_net_infer<float>(const NetGeo &, const NetDev &, const float *, const float *, const uint32_t *,
                                      float *, float *, const Scalars *, int, hipStream_t);
template void launch_net_out<double>(const NetGeo &, const NetDev &, const NetActs &, const double *, double *,
                                     float *, const Scalars *, int, hipStream_t);
template void launch_net_out<float>(const NetGeo &, const NetDev &, const NetActs &, const float *, float *, float *,
                                    const Scalars *, int, hipStream_t);

}  // namespace eg
