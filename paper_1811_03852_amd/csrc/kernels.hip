// HIP kernels (gfx950) of the BiCGStab hot path.
//
//   k_spmv      y = A x for the 7-point operator (Sec. 2, Eq. 4), fused with the FP64 partial
//               sums of the two dot products the iteration needs next.  Memory-bound.
//   k_thomas    z = T^{-1} q, T the vertical tridiagonal of A (Sec. 2, Eq. 6-7), one lane per
//               column, levels walked in registers, fused with the vector update that forms q.
//   k_update    x += alpha phat + omega shat; r = s - omega t; <rhat, r>, <r, r> partials.
//   k_finalize  fixed-order FP64 sum of the per-workgroup partials (Sec. 4: 64-bit global
//               sums) and the scalar recurrences of BiCGStab, in one workgroup.
//   k_sor_half_reg, k_sor_half
//               one red-black half-sweep of the vertical-line SOR (Sec. 2, Eq. 7).
//   k_mdot, k_maxpy, k_msum, k_vscale
//               Gram-Schmidt building blocks of FGMRES.
//
// Every floating-point sum that leaves a workgroup is FP64 and is reduced in a fixed order, so
// results are bitwise reproducible for a given grid.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "eg_internal.h"


namespace eg {

// ------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }
__device__ __forceinline__ float fp16_to_f(uint16_t b) { return static_cast<float>(__builtin_bit_cast(_Float16, b)); }

__device__ __forceinline__ bool stopped(const Scalars *sc, int mask)
{
    if (!sc || !mask) return false;
    int f = 0;
    if (sc->done) f |= STOP_DONE;
    if (sc->skip) f |= STOP_SKIP;
    if (sc->half) f |= STOP_HALF;
    return (f & mask) != 0;
}

// Sum NV doubles over the 256-thread workgroup in a fixed order; thread 0 writes `row`.
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double *row)
{
    __shared__ double sm[kWG / 64][NV];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c] += __shfl_xor(v[c], off);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) sm[wv][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = sm[0][c];
#pragma unroll
            for (int w = 1; w < kWG / 64; ++w) s += sm[w][c];
            row[c] = s;
        }
#pragma unroll
        for (int c = NV; c < kPartialCols; ++c) row[c] = 0.0;
    }
}

// Sum NV doubles over one wave in a fixed order (butterfly); lane 0 writes `row`.
template <int NV>
__device__ __forceinline__ void wave_sum_store(double (&v)[NV], double *row)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c] += __shfl_xor(v[c], off);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) row[c] = v[c];
#pragma unroll
        for (int c = NV; c < kPartialCols; ++c) row[c] = 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// k_spmv: 7-point stencil, difference form  y = m x + sum_d a_d (x - x_d)
//
// Workgroup = 4 waves; wave w of tile (bx, by) owns longitudes bx*64 + lane and the R
// consecutive latitude rows starting at (by*4 + w)*R, and walks levels k0..k1-1 of that
// strip.  x is read once per point: the vertical neighbours come from a rolling register
// window (x_{k-1}, x_k, x_{k+1}), the N/S neighbours from the same lane's other rows (two
// halo rows per level are loaded), the E/W neighbours by cross-lane shuffles (edge lanes
// load theirs, with the periodic wrap in longitude).
//
// Tiles are assigned XCD-aware: workgroups are dispatched round-robin over the 8 XCDs, so
// workgroup b processes tile (b % 8) * per_xcd + b / 8 and each XCD walks one contiguous
// range of tiles (lon-fastest order), keeping latitude-adjacent tiles in one L2.
// ------------------------------------------------------------------------------------------
enum { SPM_PLAIN = 0, SPM_DOT2 = 1, SPM_RESID = 2 };

template <typename T> __device__ __forceinline__ T ldb(const T *base, uint32_t boff)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}
template <typename T> __device__ __forceinline__ void stb(T *base, uint32_t boff, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff) = v;
}
// Streaming accesses (data touched once per kernel): non-temporal hints.  Measured on the
// 2560x1920x70 grid they raise the Thomas and SpMV rates by 5-7% over plain accesses.
template <typename T> __device__ __forceinline__ T ldn(const T *base, uint32_t boff)
{
    return __builtin_nontemporal_load(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff));
}
template <typename T> __device__ __forceinline__ void stn(T *base, uint32_t boff, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff));
}

// A coupling of row i: FP64 and FP32 sets hold it; a 16-bit set holds q with
// coupling = offset + q * scale (one offset and one power-of-two scale per direction, level and
// latitude row), rounded once to FP32 (q * scale is exact, so the fma rounds only the sum).
template <typename Tc> struct DecB;
template <> struct DecB<double> {
    __device__ static __forceinline__ double get(const double *row, uint32_t i, float, float)
    {
        return ldn(row, i * 8u);
    }
};
template <> struct DecB<float> {
    __device__ static __forceinline__ float get(const float *row, uint32_t i, float, float) { return ldn(row, i * 4u); }
};
template <> struct DecB<bf16_t> {
    __device__ static __forceinline__ float get(const bf16_t *row, uint32_t i, float s, float off)
    {
        return __builtin_fmaf(bf16_to_f(ldn(reinterpret_cast<const uint16_t *>(row), i * 2u)), s, off);
    }
};
template <> struct DecB<fp16_t> {
    __device__ static __forceinline__ float get(const fp16_t *row, uint32_t i, float s, float off)
    {
        return __builtin_fmaf(fp16_to_f(ldn(reinterpret_cast<const uint16_t *>(row), i * 2u)), s, off);
    }
};

template <typename Tv, typename Tc, int R, int MODE, typename Tout>
__global__ __launch_bounds__(kWG) void k_spmv(OpView<Tc> op, const Tv *__restrict__ x, Tout *__restrict__ y,
                                              const Tv *__restrict__ w, double *__restrict__ partials,
                                              const Scalars *__restrict__ sc, int stop_mask, int gx, int gy,
                                              int kchunk, int ntiles, int per_xcd)
{
    if (stopped(sc, stop_mask)) return;
    using V = typename CoefTraits<Tc>::val;
    constexpr bool Q = CoefTraits<Tc>::quant;
    constexpr int ND = (MODE == SPM_PLAIN) ? 0 : (MODE == SPM_DOT2 ? 2 : 3);

    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    double acc[ND > 0 ? ND : 1];
#pragma unroll
    for (int c = 0; c < (ND > 0 ? ND : 1); ++c) acc[c] = 0.0;

    if (t < ntiles) {
        const int nlon = op.nlon, nlat = op.nlat, nlev = op.nlev;
        const size_t P = op.P, n = op.n;
        const int bx = t % gx;
        const int rest = t / gx;
        const int by = rest % gy;
        const int bz = rest / gy;
        const int lane = threadIdx.x & 63;
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
        const int i = bx * 64 + lane;
        const bool iv = i < nlon;
        // lane offsets within a latitude row (everything else is a wave-uniform base)
        const uint32_t ic = iv ? i : nlon - 1;
        const uint32_t iw = (ic == 0) ? nlon - 1 : ic - 1;
        const uint32_t ie = (ic == (uint32_t)nlon - 1) ? 0 : ic + 1;
        const uint32_t xo = ic * sizeof(Tv);
        const bool needw = (lane == 0);
        const bool neede = (lane == 63) || (ic == (uint32_t)nlon - 1);
        const int j0 = (by * 4 + wv) * R;
        int jc[R];
        bool jv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            jv[r] = (j0 + r) < nlat;
            jc[r] = jv[r] ? j0 + r : nlat - 1;
        }
        const int jsh = (j0 == 0) ? 0 : ((j0 - 1 < nlat) ? j0 - 1 : nlat - 1);   // south halo row
        const int k0 = bz * kchunk;
        const int k1 = (k0 + kchunk < nlev) ? k0 + kchunk : nlev;
        auto rowx = [&](int k, int j) { return x + (size_t)k * P + (size_t)j * nlon; };

        Tv xp[R], xc[R], xn[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xc[r] = ldb(rowx(k0, jc[r]), xo);
            xp[r] = (k0 > 0) ? ldb(rowx(k0 - 1, jc[r]), xo) : xc[r];
        }
        for (int k = k0; k < k1; ++k) {
            const bool up = (k + 1) < nlev;
#pragma unroll
            for (int r = 0; r < R; ++r) xn[r] = up ? ldb(rowx(k + 1, jc[r]), xo) : xc[r];
            const Tv hs = (j0 > 0) ? ldb(rowx(k, jsh), xo) : xc[0];
            const Tv hn = (j0 + R < nlat) ? ldb(rowx(k, j0 + R), xo) : xc[R - 1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const size_t rowoff = (size_t)k * P + (size_t)jc[r] * nlon;   // wave-uniform
                const Tv *xr_row = x + rowoff;
                const Tv xr = xc[r];
                Tv xw = __shfl_up(xr, 1);
                Tv xe = __shfl_down(xr, 1);
                if (needw) xw = ldb(xr_row, iw * (uint32_t)sizeof(Tv));
                if (neede) xe = ldb(xr_row, ie * (uint32_t)sizeof(Tv));
                const Tv xs = (r == 0) ? hs : xc[r - 1];
                const Tv xnn = (r == R - 1) ? hn : xc[r + 1];
                float s0 = 1.f, s1 = 1.f, s2 = 1.f, s3 = 1.f, s4 = 1.f, s5 = 1.f;
                float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f, f4 = 0.f, f5 = 0.f;
                if constexpr (Q) {
                    // the row's six scales and six offsets: one wave-uniform 64-byte record
                    const float4 *qr = reinterpret_cast<const float4 *>(op.qs + ((size_t)k * nlat + jc[r]) * kQsStride);
                    const float4 q0 = qr[0], q1 = qr[1], o0 = qr[2], o1 = qr[3];
                    s0 = q0.x;
                    s1 = q0.y;
                    s2 = q0.z;
                    s3 = q0.w;
                    s4 = q1.x;
                    s5 = q1.y;
                    f0 = o0.x;
                    f1 = o0.y;
                    f2 = o0.z;
                    f3 = o0.w;
                    f4 = o1.x;
                    f5 = o1.y;
                }
                const Tc *arow = op.a + rowoff;
                const V aW = DecB<Tc>::get(arow, ic, s0, f0);
                const V aE = DecB<Tc>::get(arow + n, ic, s1, f1);
                const V aS = DecB<Tc>::get(arow + 2 * n, ic, s2, f2);
                const V aN = DecB<Tc>::get(arow + 3 * n, ic, s3, f3);
                const V aD = DecB<Tc>::get(arow + 4 * n, ic, s4, f4);
                const V aU = DecB<Tc>::get(arow + 5 * n, ic, s5, f5);
                const V mm = ldn(op.m + rowoff, ic * (uint32_t)sizeof(V));
                Tv yv = mm * xr;
                yv += aW * (xr - xw);
                yv += aE * (xr - xe);
                yv += aS * (xr - xs);
                yv += aN * (xr - xnn);
                yv += aD * (xr - xp[r]);
                yv += aU * (xr - xn[r]);
                if (iv && jv[r]) {
                    if constexpr (MODE == SPM_RESID) {
                        const double bb = static_cast<double>(ldn(w + rowoff, xo));
                        const double rv = bb - static_cast<double>(yv);
                        const Tout ro = static_cast<Tout>(rv);
                        if (y) stn(y + rowoff, ic * (uint32_t)sizeof(Tout), ro);
                        acc[0] += rv * rv;
                        acc[1] += bb * bb;
                        acc[2] += static_cast<double>(ro) * static_cast<double>(ro);
                    } else {
                        stn(y + rowoff, ic * (uint32_t)sizeof(Tout), static_cast<Tout>(yv));
                        if constexpr (MODE == SPM_DOT2) {
                            acc[0] += static_cast<double>(ldn(w + rowoff, xo)) * static_cast<double>(yv);
                            acc[1] += static_cast<double>(yv) * static_cast<double>(yv);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                xp[r] = xc[r];
                xc[r] = xn[r];
            }
        }
    }
    if constexpr (ND > 0) block_sum_store<ND>(acc, partials + (long)b * kPartialCols);
}

struct SpmvGrid {
    int gx, gy, gz, kchunk, ntiles, per_xcd, nblocks;
};

template <int R>
static SpmvGrid spmv_grid(int nlon, int nlat, int nlev)
{
    SpmvGrid g;
    g.gx = (nlon + 63) / 64;
    g.gy = (nlat + 4 * R - 1) / (4 * R);
    // split the level march when the horizontal tiling alone cannot fill the chip
    const int tiles2d = g.gx * g.gy;
    int chunks = 1;
    while (tiles2d * chunks < 2048 && chunks < nlev) chunks *= 2;
    if (chunks > nlev) chunks = nlev;
    g.kchunk = (nlev + chunks - 1) / chunks;
    g.gz = (nlev + g.kchunk - 1) / g.kchunk;
    g.ntiles = tiles2d * g.gz;
    g.per_xcd = (g.ntiles + 7) / 8;
    g.nblocks = g.per_xcd * 8;
    return g;
}

constexpr int kSpmvRows = 2;   // latitude rows per thread

constexpr int kUpdateMaxBlocks = 32768;   // most workgroups of the vector-update kernels

int partial_rows_needed(int nlon, int nlat, int nlev)
{
    const long P = (long)nlon * nlat;
    long rows = spmv_grid<kSpmvRows>(nlon, nlat, nlev).nblocks;
    rows = std::max(rows, (P + 63) / 64);         // thomas(S): one row per wave of columns
    rows = std::max(rows, (long)kUpdateMaxBlocks);   // elementwise kernels (the update the most)
    return (int)rows;
}

template <typename Tv, typename Tc>
int launch_spmv_impl(const OpView<Tc> &op, const Tv *x, Tv *y, const Tv *w, int mode, double *partials,
                     const Scalars *sc, int stop_mask, hipStream_t s)
{
    constexpr int R = kSpmvRows;
    SpmvGrid g = spmv_grid<R>(op.nlon, op.nlat, op.nlev);
    if (mode == SP_DOT2)
        hipLaunchKernelGGL((k_spmv<Tv, Tc, R, SPM_DOT2, Tv>), dim3(g.nblocks), dim3(kWG), 0, s, op, x, y, w, partials,
                           sc, stop_mask, g.gx, g.gy, g.kchunk, g.ntiles, g.per_xcd);
    else
        hipLaunchKernelGGL((k_spmv<Tv, Tc, R, SPM_PLAIN, Tv>), dim3(g.nblocks), dim3(kWG), 0, s, op, x, y, w,
                           partials, sc, stop_mask, g.gx, g.gy, g.kchunk, g.ntiles, g.per_xcd);
    return mode == SP_DOT2 ? g.nblocks : 0;
}

template <typename Tv, typename Tc>
void launch_spmv(const OpView<Tc> &op, const Tv *x, Tv *y, const Tv *w, int mode, double *partials, int *nrows,
                 const Scalars *sc, int stop_mask, hipStream_t s)
{
    int rows = launch_spmv_impl<Tv, Tc>(op, x, y, w, mode, partials, sc, stop_mask, s);
    if (nrows) *nrows = rows;
}

template <typename Tout>
void launch_residual(const OpView<double> &op, const double *b, const double *x, Tout *r, double *partials,
                     int *nrows, hipStream_t s)
{
    constexpr int R = kSpmvRows;
    SpmvGrid g = spmv_grid<R>(op.nlon, op.nlat, op.nlev);
    hipLaunchKernelGGL((k_spmv<double, double, R, SPM_RESID, Tout>), dim3(g.nblocks), dim3(kWG), 0, s, op, x, r, b,
                       partials, nullptr, 0, g.gx, g.gy, g.kchunk, g.ntiles, g.per_xcd);
    if (nrows) *nrows = g.nblocks;
}

// ------------------------------------------------------------------------------------------
// Thomas factors of T = tridiag(-aD, C, -aU), computed once per operator (the paper notes the
// LU factorisation of T can be precomputed per horizontal point).  With
//   den_k = C_k - aD_k aU_{k-1} / den_{k-1},  inv_k = 1 / den_k,
//   l_k = aD_k inv_{k-1}  (l_0 = 0),          c_k = aU_k inv_k,
// the solve is  w_k = q_k + l_k w_{k-1}  (forward)  and  z_k = inv_k w_k + c_k z_{k+1}  (back).
// den_k is evaluated through the excess e_k = den_k - aU_k = g_k + aD_k e_{k-1} / den_{k-1},
// g = m + W + E + S + N, in FP64: every term is non-negative, so no cancellation occurs even
// where the horizontal coupling is tiny next to the vertical one.  f[3][n] = (l, inv, c).
// ------------------------------------------------------------------------------------------
template <typename Tf>
__global__ __launch_bounds__(kWG) void k_tri_factor(const double *__restrict__ a64, const double *__restrict__ m64,
                                                    int nlon, int nlat, int nlev, Tf *__restrict__ f)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    const long col = (long)blockIdx.x * kWG + threadIdx.x;
    if (col >= P) return;
    double ratio = 0.0, inv_prev = 0.0;
    for (int k = 0; k < nlev; ++k) {
        const long c = col + (long)k * P;
        const double g = m64[c] + (((a64[c] + a64[n + c]) + a64[2 * n + c]) + a64[3 * n + c]);
        const double aD = a64[4 * n + c], aU = a64[5 * n + c];
        const double e = g + aD * ratio;
        const double den = e + aU;
        const double inv = 1.0 / den;
        f[c] = static_cast<Tf>(aD * inv_prev);
        f[n + c] = static_cast<Tf>(inv);
        f[2 * n + c] = static_cast<Tf>(aU * inv);
        ratio = e * inv;
        inv_prev = inv;
    }
}

template <typename Tf>
void launch_tri_factor(const double *a64, const double *m64, int nlon, int nlat, int nlev, Tf *f, hipStream_t s)
{
    const long P = (long)nlon * nlat;
    hipLaunchKernelGGL((k_tri_factor<Tf>), dim3((unsigned)((P + kWG - 1) / kWG)), dim3(kWG), 0, s, a64, m64, nlon,
                       nlat, nlev, f);
}

// ------------------------------------------------------------------------------------------
// k_thomas: z = T^{-1} q per column from the precomputed factors.
//
// One lane per column; lane -> column col = j*nlon + i, so each level's load is a contiguous
// run of the plane.  NL > 0: exactly NL levels, the forward values w_k held in registers.
// NL == 0: any nlev, w_k parked in z between the sweeps.
//
// Prologues: TH_PLAIN  q read from `q`;
//            TH_P      q = r + beta (p - omega v), stored to p (on a restart q = r and rhat = r);
//            TH_S      q = r - alpha v, stored to s (passed as `p`), ||q||^2 partial.
// CM: z is written in the colour-major order of the line-SOR kernels (index
// colour * n/2 + k * P/2 + j * nlon/2 + i/2, colour = (i + j) & 1, nlon even) and q is also
// stored there, to qcm: the start of a line-SOR application (both in one pass).
// ------------------------------------------------------------------------------------------
// One wave per workgroup: with the register-resident columns (up to 199 VGPRs in FP64, two
// waves per SIMD) a finished wave is replaced at once on its own SIMD instead of waiting for
// the other waves of a four-wave workgroup; 5.66 instead of 5.26 TB/s for TH_P at
// 2560x1920x70 in FP64.
constexpr int kTriWG = 64;

template <typename Tv, int NL, int MODE, bool CM, int PF>
__device__ __forceinline__ void thomas_body(TriView<Tv> tv, const Tv *__restrict__ q, Tv *__restrict__ z,
                                            const Tv *__restrict__ r, Tv *__restrict__ p, const Tv *__restrict__ v,
                                            Tv *__restrict__ rhat, double *__restrict__ partials,
                                            const Scalars *__restrict__ sc, int stop_mask, Tv *__restrict__ qcm,
                                            int nlon)
{
    if (stopped(sc, stop_mask)) return;
    const long P = tv.P, n = tv.n;
    const int nlev = (NL > 0) ? NL : tv.nlev;
    const long col = (long)blockIdx.x * kTriWG + threadIdx.x;
    const bool act = col < P;
    // 32-bit lane offset within a level plane; per-level bases below are wave-uniform
    const unsigned cu = static_cast<unsigned>(act ? col : P - 1);
    // colour-major element index of this column's level 0 (CM only) and the level stride
    long cm0 = 0;
    if constexpr (CM) {
        const int i = (int)(cu % (unsigned)nlon), j = (int)(cu / (unsigned)nlon);
        cm0 = (long)((i + j) & 1) * (n / 2) + (long)j * (nlon / 2) + i / 2;
    }
    const long P2 = P / 2;
    const Tv *lf = tv.f;
    const Tv *invf = tv.f + n;
    const Tv *cf = tv.f + 2 * n;
    Tv beta = 0, omega = 0, alpha = 0;
    int fresh = 0;
    if constexpr (MODE == TH_P) {
        fresh = sc->fresh;
        // on the register path a restart iteration is TH_PF's (a separate kernel keeps this
        // one's forward sweep free of the restart variant: 3.9 instead of 4.2 ms at 2560x1920x70)
        if constexpr (NL > 0)
            if (fresh) return;
        beta = static_cast<Tv>(sc->beta);
        omega = static_cast<Tv>(sc->omega);
    }
    if constexpr (MODE == TH_PF)
        if (!sc->fresh) return;
    if constexpr (MODE == TH_S) alpha = static_cast<Tv>(sc->alpha);
    double acc[1] = {0.0};
    auto lv = [&](auto *base, int k) { return base + (size_t)k * (size_t)P; };

    if constexpr (NL > 0) {
        // Register path (the launcher guarantees P % kTriWG == 0, so every lane owns a column,
        // and n * sizeof(Tv) < 2^32, so level offsets fit 32-bit byte offsets from the
        // wave-uniform array bases).  Software pipeline: the loads of level k + PF are issued
        // while level k is computed, into a ring of PF register slots; the scheduling fences
        // stop the compiler from hoisting all levels' loads (which would exhaust registers).
        const uint32_t step = static_cast<uint32_t>(P * sizeof(Tv));
        const uint32_t bo0 = cu * static_cast<uint32_t>(sizeof(Tv));
        const uint32_t cstep = static_cast<uint32_t>(P2 * sizeof(Tv));
        const uint32_t cbo0 = static_cast<uint32_t>(cm0 * (long)sizeof(Tv));
        auto ld = [](const Tv *base, uint32_t bo) { return ldn(base, bo); };
        auto st = [](Tv *base, uint32_t bo, Tv val) { stn(base, bo, val); };
        Tv w[NL];
        {
            Tv b0[PF], b1[PF], b2[PF], bl[PF];
            uint32_t bl_off = bo0;   // next level to load
            auto issue = [&](int sl) {
                if constexpr (MODE == TH_PLAIN) {
                    b0[sl] = ld(q, bl_off);
                } else if constexpr (MODE == TH_P) {
                    b0[sl] = ld(r, bl_off);
                    b1[sl] = ld(p, bl_off);
                    b2[sl] = ld(v, bl_off);
                } else if constexpr (MODE == TH_PF) {
                    b0[sl] = ld(r, bl_off);
                } else {
                    b0[sl] = ld(r, bl_off);
                    b2[sl] = ld(v, bl_off);
                }
                bl[sl] = ld(lf, bl_off);
                bl_off += step;
            };
#pragma unroll
            for (int k = 0; k < PF && k < NL; ++k) issue(k);
            uint32_t bo = bo0;
            uint32_t cbo = cbo0;
            Tv wprev = 0;
            double ss = 0.0;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int sl = k % PF;
                Tv qk;
                if constexpr (MODE == TH_PLAIN) {
                    qk = b0[sl];
                } else if constexpr (MODE == TH_P) {
                    qk = b0[sl] + beta * (b1[sl] - omega * b2[sl]);
                    st(p, bo, qk);
                } else if constexpr (MODE == TH_PF) {
                    qk = b0[sl];
                    st(rhat, bo, qk);
                    st(p, bo, qk);
                } else {
                    qk = b0[sl] - alpha * b2[sl];
                    st(p, bo, qk);
                    ss = fma(static_cast<double>(qk), static_cast<double>(qk), ss);
                    // empty asm: pins the accumulation to this level (otherwise the compiler
                    // sinks all the FP64 products to the end and keeps NL values live)
                    asm volatile("" : "+v"(ss));
                }
                if constexpr (CM) {
                    st(qcm, cbo, qk);
                    cbo += cstep;
                }
                w[k] = qk + bl[sl] * wprev;
                wprev = w[k];
                bo += step;
                if (k + PF < NL) issue(sl);
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (MODE == TH_S) acc[0] = ss;
        }
        Tv bi[PF], bc[PF];
        uint32_t bl_off = bo0 + static_cast<uint32_t>(NL - 1) * step;
#pragma unroll
        for (int j = 0; j < PF && j < NL; ++j) {
            bi[j] = ld(invf, bl_off);
            bc[j] = ld(cf, bl_off);
            bl_off -= step;
        }
        uint32_t bo = CM ? cbo0 + static_cast<uint32_t>(NL - 1) * cstep : bo0 + static_cast<uint32_t>(NL - 1) * step;
        Tv zz = 0;
#pragma unroll
        for (int k = NL - 1; k >= 0; --k) {
            const int sl = (NL - 1 - k) % PF;
            zz = bi[sl] * w[k] + bc[sl] * zz;
            st(z, bo, zz);
            bo -= CM ? cstep : step;
            if (k - PF >= 0) {
                bi[sl] = ld(invf, bl_off);
                bc[sl] = ld(cf, bl_off);
                bl_off -= step;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        // z index of level k (the forward values are parked there between the sweeps)
        auto zi = [&](int k) -> long { return CM ? cm0 + (long)k * P2 : (long)cu + (long)k * P; };
        Tv wprev = 0;
        for (int k = 0; k < nlev; ++k) {
            Tv qk;
            if constexpr (MODE == TH_PLAIN) {
                qk = lv(q, k)[cu];
            } else if constexpr (MODE == TH_P) {
                const Tv rk = lv(r, k)[cu];
                if (fresh) {
                    qk = rk;
                    if (act) lv(rhat, k)[cu] = rk;
                } else {
                    qk = rk + beta * (lv(p, k)[cu] - omega * lv(v, k)[cu]);
                }
                if (act) lv(p, k)[cu] = qk;
            } else {
                qk = lv(r, k)[cu] - alpha * lv(v, k)[cu];
                if (act) {
                    lv(p, k)[cu] = qk;
                    acc[0] += static_cast<double>(qk) * static_cast<double>(qk);
                }
            }
            if constexpr (CM)
                if (act) qcm[cm0 + (long)k * P2] = qk;
            wprev = qk + lv(lf, k)[cu] * wprev;
            if (act) z[zi(k)] = wprev;
        }
        if (act) {
            Tv zz = 0;
            for (int k = nlev - 1; k >= 0; --k) {
                zz = lv(invf, k)[cu] * z[zi(k)] + lv(cf, k)[cu] * zz;
                z[zi(k)] = zz;
            }
        }
    }
    if constexpr (MODE == TH_S) wave_sum_store<1>(acc, partials + (long)blockIdx.x * kPartialCols);
}

template <typename Tv, int NL, int MODE, bool CM, int PF = 8>
__global__ __launch_bounds__(kTriWG) void k_thomas(TriView<Tv> tv, const Tv *__restrict__ q, Tv *__restrict__ z,
                                                const Tv *__restrict__ r, Tv *__restrict__ p,
                                                const Tv *__restrict__ v, Tv *__restrict__ rhat,
                                                double *__restrict__ partials, const Scalars *__restrict__ sc,
                                                int stop_mask, Tv *__restrict__ qcm, int nlon)
{
    thomas_body<Tv, NL, MODE, CM, PF>(tv, q, z, r, p, v, rhat, partials, sc, stop_mask, qcm, nlon);
}

// FP32 vectors, two adjacent columns per lane: every load and store moves 8 bytes per lane (512
// per wave, as in FP64); the same arithmetic per column, so z is bitwise the one-column
// kernel's (TH_S sums ||s||^2 over the lane's two columns).  Register path only; the launcher
// guarantees P % (2 kTriWG) == 0, an even nlon and n * 4 < 2^32.  TH_P at 2560x1920x70:
// 5.50 against 5.14 TB/s with one column per lane (isolated kernels).
typedef float f2v __attribute__((ext_vector_type(2)));
template <int NL, int MODE, bool CM, int PF>
__device__ __forceinline__ void thomas_body_pair(TriView<float> tv, const float *__restrict__ q,
                                                 float *__restrict__ z, const float *__restrict__ r,
                                                 float *__restrict__ p, const float *__restrict__ v,
                                                 float *__restrict__ rhat, double *__restrict__ partials,
                                                 const Scalars *__restrict__ sc, int stop_mask,
                                                 float *__restrict__ qcm, int nlon)
{
    if (stopped(sc, stop_mask)) return;
    const long P = tv.P, n = tv.n;
    const uint32_t u = blockIdx.x * kTriWG + threadIdx.x;   // columns 2u and 2u + 1 of the plane
    float beta = 0, omega = 0, alpha = 0;
    if constexpr (MODE == TH_P) {
        if (sc->fresh) return;   // a restart iteration is TH_PF's
        beta = static_cast<float>(sc->beta);
        omega = static_cast<float>(sc->omega);
    }
    if constexpr (MODE == TH_PF)
        if (!sc->fresh) return;
    if constexpr (MODE == TH_S) alpha = static_cast<float>(sc->alpha);
    const uint32_t step = static_cast<uint32_t>(P * 4);
    const uint32_t bo0 = u * 8u;
    // colour-major element offsets of the two columns (same row, i even, so opposite colours
    // and the same index within the colour)
    uint32_t ca0 = 0, cb0 = 0;
    const uint32_t cstep = static_cast<uint32_t>(P / 2 * 4);
    if constexpr (CM) {
        const uint32_t c0 = 2 * u;
        const int i = (int)(c0 % (uint32_t)nlon), j = (int)(c0 / (uint32_t)nlon);
        const long within = (long)j * (nlon / 2) + i / 2;
        const long colour = (i + j) & 1;
        ca0 = static_cast<uint32_t>((colour * (n / 2) + within) * 4);
        cb0 = static_cast<uint32_t>(((colour ^ 1) * (n / 2) + within) * 4);
    }
    const float *lf = tv.f;
    const float *invf = tv.f + n;
    const float *cf = tv.f + 2 * n;
    auto ld = [](const float *base, uint32_t bo) { return ldn(reinterpret_cast<const f2v *>(base), bo); };
    auto st = [](float *base, uint32_t bo, f2v val) { stn(reinterpret_cast<f2v *>(base), bo, val); };
    double acc[1] = {0.0};
    f2v w[NL];
    {
        f2v b0[PF], b1[PF], b2[PF], bl[PF];
        uint32_t bl_off = bo0;
        auto issue = [&](int sl) {
            if constexpr (MODE == TH_PLAIN) {
                b0[sl] = ld(q, bl_off);
            } else if constexpr (MODE == TH_P) {
                b0[sl] = ld(r, bl_off);
                b1[sl] = ld(p, bl_off);
                b2[sl] = ld(v, bl_off);
            } else if constexpr (MODE == TH_PF) {
                b0[sl] = ld(r, bl_off);
            } else {
                b0[sl] = ld(r, bl_off);
                b2[sl] = ld(v, bl_off);
            }
            bl[sl] = ld(lf, bl_off);
            bl_off += step;
        };
#pragma unroll
        for (int k = 0; k < PF && k < NL; ++k) issue(k);
        uint32_t bo = bo0, ca = ca0, cb = cb0;
        f2v wprev = {0.f, 0.f};
        double ss = 0.0;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int sl = k % PF;
            f2v qk;
            if constexpr (MODE == TH_PLAIN) {
                qk = b0[sl];
            } else if constexpr (MODE == TH_P) {
                qk = b0[sl] + beta * (b1[sl] - omega * b2[sl]);
                st(p, bo, qk);
            } else if constexpr (MODE == TH_PF) {
                qk = b0[sl];
                st(rhat, bo, qk);
                st(p, bo, qk);
            } else {
                qk = b0[sl] - alpha * b2[sl];
                st(p, bo, qk);
                ss = fma(static_cast<double>(qk.x), static_cast<double>(qk.x), ss);
                ss = fma(static_cast<double>(qk.y), static_cast<double>(qk.y), ss);
                asm volatile("" : "+v"(ss));
            }
            if constexpr (CM) {
                stn(qcm, ca, qk.x);
                stn(qcm, cb, qk.y);
                ca += cstep;
                cb += cstep;
            }
            w[k] = qk + bl[sl] * wprev;
            wprev = w[k];
            bo += step;
            if (k + PF < NL) issue(sl);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (MODE == TH_S) acc[0] = ss;
    }
    f2v bi[PF], bc[PF];
    uint32_t bl_off = bo0 + static_cast<uint32_t>(NL - 1) * step;
#pragma unroll
    for (int j = 0; j < PF && j < NL; ++j) {
        bi[j] = ld(invf, bl_off);
        bc[j] = ld(cf, bl_off);
        bl_off -= step;
    }
    uint32_t bo = bo0 + static_cast<uint32_t>(NL - 1) * step;
    uint32_t ca = ca0 + static_cast<uint32_t>(NL - 1) * cstep, cb = cb0 + static_cast<uint32_t>(NL - 1) * cstep;
    f2v zz = {0.f, 0.f};
#pragma unroll
    for (int k = NL - 1; k >= 0; --k) {
        const int sl = (NL - 1 - k) % PF;
        zz = bi[sl] * w[k] + bc[sl] * zz;
        if constexpr (CM) {
            stn(z, ca, zz.x);
            stn(z, cb, zz.y);
            ca -= cstep;
            cb -= cstep;
        } else {
            st(z, bo, zz);
            bo -= step;
        }
        if (k - PF >= 0) {
            bi[sl] = ld(invf, bl_off);
            bc[sl] = ld(cf, bl_off);
            bl_off -= step;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (MODE == TH_S) wave_sum_store<1>(acc, partials + (long)blockIdx.x * kPartialCols);
}

template <int NL, int MODE, bool CM, int PF = 8>
__global__ __launch_bounds__(kTriWG) void k_thomas_pair(TriView<float> tv, const float *__restrict__ q,
                                                     float *__restrict__ z, const float *__restrict__ r,
                                                     float *__restrict__ p, const float *__restrict__ v,
                                                     float *__restrict__ rhat, double *__restrict__ partials,
                                                     const Scalars *__restrict__ sc, int stop_mask,
                                                     float *__restrict__ qcm, int nlon)
{
    thomas_body_pair<NL, MODE, CM, PF>(tv, q, z, r, p, v, rhat, partials, sc, stop_mask, qcm, nlon);
}

// Deep columns in FP64 (140 levels: 280 registers of forward values): one wave per SIMD, so the
// compiler may use the whole register file (architectural and accumulation registers) and keep
// 24 levels of loads in flight.  5.46 TB/s at 1280x960x140 against 3.95 TB/s for parking the
// forward values in memory (the generic path, +16 B per point).
constexpr int kDeepPF = 24;
template <typename Tv, int NL, int MODE, bool CM>
__global__ __launch_bounds__(kTriWG) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_thomas_deep(
    TriView<Tv> tv, const Tv *__restrict__ q, Tv *__restrict__ z, const Tv *__restrict__ r, Tv *__restrict__ p,
    const Tv *__restrict__ v, Tv *__restrict__ rhat, double *__restrict__ partials, const Scalars *__restrict__ sc,
    int stop_mask, Tv *__restrict__ qcm, int nlon)
{
    thomas_body<Tv, NL, MODE, CM, kDeepPF>(tv, q, z, r, p, v, rhat, partials, sc, stop_mask, qcm, nlon);
}

template <typename Tv, int NL, bool CM, bool DEEP = false, bool PAIR = false>
static int thomas_dispatch_mode(const TriView<Tv> &tv, const Tv *q, Tv *z, int mode, const Tv *r, Tv *p,
                                const Tv *v, Tv *rhat, double *partials, const Scalars *sc, hipStream_t s,
                                int stop_mask, Tv *qcm, int nlon)
{
    const int nb = (int)((tv.P / (PAIR ? 2 : 1) + kTriWG - 1) / kTriWG);
    auto launch = [&](auto mode_c, int mask) {
        constexpr int M = decltype(mode_c)::value;
        if constexpr (PAIR)
            hipLaunchKernelGGL((k_thomas_pair<NL, M, CM>), dim3(nb), dim3(kTriWG), 0, s, tv, q, z, r, p, v, rhat,
                               partials, sc, mask, qcm, nlon);
        else if constexpr (DEEP)
            hipLaunchKernelGGL((k_thomas_deep<Tv, NL, M, CM>), dim3(nb), dim3(kTriWG), 0, s, tv, q, z, r, p, v, rhat,
                               partials, sc, mask, qcm, nlon);
        else
            hipLaunchKernelGGL((k_thomas<Tv, NL, M, CM>), dim3(nb), dim3(kTriWG), 0, s, tv, q, z, r, p, v, rhat,
                               partials, sc, mask, qcm, nlon);
    };
    switch (mode) {
    case TH_P:
        if constexpr (NL > 0) launch(std::integral_constant<int, TH_PF>{}, STOP_DONE);
        launch(std::integral_constant<int, TH_P>{}, STOP_DONE);
        return 0;
    case TH_S:
        launch(std::integral_constant<int, TH_S>{}, STOP_DONE | STOP_SKIP);
        return nb;
    default:
        launch(std::integral_constant<int, TH_PLAIN>{}, stop_mask);
        return 0;
    }
}

template <typename Tv, bool CM>
static int thomas_dispatch(const TriView<Tv> &tv, const Tv *q, Tv *z, int mode, const Tv *r, Tv *p, const Tv *v,
                           Tv *rhat, double *partials, const Scalars *sc, hipStream_t s, int stop_mask, Tv *qcm,
                           int nlon)
{
    // Register-resident forward values for the level counts in use, on grids whose columns
    // fill whole workgroups and whose arrays are addressable with 32-bit byte offsets; any
    // other grid takes the generic path.
    const bool reg = (tv.P % kTriWG == 0) && ((unsigned long)tv.n * sizeof(Tv) < (1ul << 32));
    if constexpr (sizeof(Tv) == 4) {
        // FP32: two columns per lane where the plane fills whole waves of column pairs (and, for
        // the colour-major output, the pairs lie within a latitude row)
        const bool pair = reg && tv.P % (2 * kTriWG) == 0 && (!CM || nlon % 2 == 0);
        if (pair && tv.nlev == 20)
            return thomas_dispatch_mode<Tv, 20, CM, false, true>(tv, q, z, mode, r, p, v, rhat, partials, sc, s,
                                                                  stop_mask, qcm, nlon);
        if (pair && tv.nlev == 70)
            return thomas_dispatch_mode<Tv, 70, CM, false, true>(tv, q, z, mode, r, p, v, rhat, partials, sc, s,
                                                                  stop_mask, qcm, nlon);
    }
    if (reg && tv.nlev == 20)
        return thomas_dispatch_mode<Tv, 20, CM>(tv, q, z, mode, r, p, v, rhat, partials, sc, s, stop_mask, qcm, nlon);
    if (reg && tv.nlev == 70)
        return thomas_dispatch_mode<Tv, 70, CM>(tv, q, z, mode, r, p, v, rhat, partials, sc, s, stop_mask, qcm, nlon);
    if (reg && tv.nlev == 140) {
        if constexpr (sizeof(Tv) == 4)
            return thomas_dispatch_mode<Tv, 140, CM>(tv, q, z, mode, r, p, v, rhat, partials, sc, s, stop_mask, qcm,
                                                     nlon);
        else
            return thomas_dispatch_mode<Tv, 140, CM, true>(tv, q, z, mode, r, p, v, rhat, partials, sc, s, stop_mask,
                                                           qcm, nlon);
    }
    return thomas_dispatch_mode<Tv, 0, CM>(tv, q, z, mode, r, p, v, rhat, partials, sc, s, stop_mask, qcm, nlon);
}

template <typename Tv>
void launch_thomas(const TriView<Tv> &tv, const Tv *q, Tv *z, int mode, const Tv *r, Tv *p, const Tv *v, Tv *rhat,
                   double *partials, int *nrows, const Scalars *sc, hipStream_t s, int stop_mask)
{
    const int rows = thomas_dispatch<Tv, false>(tv, q, z, mode, r, p, v, rhat, partials, sc, s, stop_mask, nullptr, 0);
    if (nrows) *nrows = rows;
}

template <typename Tv>
void launch_thomas_cm(const TriView<Tv> &tv, int nlon, const Tv *q, Tv *zcm, Tv *qcm, int mode, const Tv *r, Tv *p,
                      const Tv *v, Tv *rhat, double *partials, int *nrows, const Scalars *sc, hipStream_t s,
                      int stop_mask)
{
    const int rows = thomas_dispatch<Tv, true>(tv, q, zcm, mode, r, p, v, rhat, partials, sc, s, stop_mask, qcm, nlon);
    if (nrows) *nrows = rows;
}

// ------------------------------------------------------------------------------------------
// k_update: end of a BiCGStab iteration.
//   full step    x += alpha phat + omega shat; r = s - omega t; partials <rhat, r>, <r, r>
//   half step    x += alpha phat                      (converged at s)
//   omega = 0    x += alpha phat; r = s; partial <r, r>   (restart follows)
// 16-byte vector accesses (double2 / float4); the n % VEC tail is done by workgroup 0.
// ------------------------------------------------------------------------------------------
// 16-byte vectors for the elementwise kernels
template <typename T> struct Vec16;
template <> struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};
template <> struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <typename T> __device__ __forceinline__ typename Vec16<T>::type ldv(const T *p, long i)
{
    using VT = typename Vec16<T>::type;
    return __builtin_nontemporal_load(reinterpret_cast<const VT *>(p) + i);
}
template <typename T> __device__ __forceinline__ void stv(T *p, long i, typename Vec16<T>::type v)
{
    using VT = typename Vec16<T>::type;
    __builtin_nontemporal_store(v, reinterpret_cast<VT *>(p) + i);
}

template <typename Tv>
__device__ __forceinline__ void update_one(int mode, Tv alpha, Tv omega, Tv &x, Tv ph, Tv sh, Tv s, Tv t, Tv &r,
                                           Tv rh, double (&acc)[2])
{
    if (mode == 1) {
        x = x + alpha * ph;
    } else if (mode == 2) {
        x = x + alpha * ph;
        r = s;
        acc[1] += static_cast<double>(s) * static_cast<double>(s);
    } else {
        x = x + alpha * ph + omega * sh;
        r = s - omega * t;
        acc[0] += static_cast<double>(rh) * static_cast<double>(r);
        acc[1] += static_cast<double>(r) * static_cast<double>(r);
    }
}

template <typename Tv>
__global__ __launch_bounds__(kWG) void k_update(long n, Tv *__restrict__ x, const Tv *__restrict__ ph,
                                                const Tv *__restrict__ sh, const Tv *__restrict__ s,
                                                const Tv *__restrict__ t, Tv *__restrict__ r,
                                                const Tv *__restrict__ rhat, double *__restrict__ partials,
                                                const Scalars *__restrict__ sc)
{
    if (sc->done || sc->skip) return;
    const Tv alpha = static_cast<Tv>(sc->alpha);
    const Tv omega = static_cast<Tv>(sc->omega);
    const int mode = sc->half ? 1 : (sc->wbd ? 2 : 0);
    using VT = typename Vec16<Tv>::type;
    constexpr int V = Vec16<Tv>::N;
    double acc[2] = {0.0, 0.0};
    const long nv = n / V;
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < nv; i += stride) {
        VT xv = ldv(x, i);
        const VT pv = ldv(ph, i);
        VT sv = {}, hv = {}, tv = {}, rv = {}, qv = {};
        if (mode != 1) sv = ldv(s, i);
        if (mode == 0) {
            hv = ldv(sh, i);
            tv = ldv(t, i);
            qv = ldv(rhat, i);
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
            Tv xe = xv[e], re = 0;
            update_one<Tv>(mode, alpha, omega, xe, pv[e], hv[e], sv[e], tv[e], re, qv[e], acc);
            xv[e] = xe;
            rv[e] = re;
        }
        stv(x, i, xv);
        if (mode != 1) stv(r, i, rv);
    }
    if (blockIdx.x == 0)
        for (long i = nv * V + threadIdx.x; i < n; i += kWG) {
            Tv xi = x[i], ri = 0;
            const Tv si = (mode != 1) ? s[i] : Tv(0);
            const Tv hi = (mode == 0) ? sh[i] : Tv(0), ti = (mode == 0) ? t[i] : Tv(0);
            const Tv qi = (mode == 0) ? rhat[i] : Tv(0);
            update_one<Tv>(mode, alpha, omega, xi, ph[i], hi, si, ti, ri, qi, acc);
            x[i] = xi;
            if (mode != 1) r[i] = ri;
        }
    block_sum_store<2>(acc, partials + (long)blockIdx.x * kPartialCols);
}

// The paper's mixed-precision update (Sec. 3 and Sec. 4): the solution stays FP64 and is
// updated every iteration from the FP32 search directions with the FP64 scalars; the
// residual recurrence stays FP32.  Same modes as k_update (full step, half step, half step
// after a t = 0 breakdown).
// X32: the solution is held in 32 bits as well (rounded after every update): the all-32-bit
// solver the paper compares with the 64-bit one in its toy model (Sec. 4, Fig. 1)
template <bool X32>
__global__ __launch_bounds__(kWG) void k_update_mp(long n, double *__restrict__ x, const float *__restrict__ ph,
                                                   const float *__restrict__ sh, const float *__restrict__ s,
                                                   const float *__restrict__ t, float *__restrict__ r,
                                                   const float *__restrict__ rhat, double *__restrict__ partials,
                                                   const Scalars *__restrict__ sc)
{
    if (sc->done || sc->skip) return;
    const double alpha = sc->alpha, omega = sc->omega;
    const float omega32 = static_cast<float>(omega);
    const int mode = sc->half ? 1 : (sc->wbd ? 2 : 0);
    double acc[2] = {0.0, 0.0};
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        double xi = x[i] + alpha * static_cast<double>(ph[i]);
        if (mode == 2) {
            const float si = s[i];
            r[i] = si;
            acc[1] += static_cast<double>(si) * static_cast<double>(si);
        } else if (mode == 0) {
            xi += omega * static_cast<double>(sh[i]);
            const float ri = s[i] - omega32 * t[i];
            r[i] = ri;
            acc[0] += static_cast<double>(rhat[i]) * static_cast<double>(ri);
            acc[1] += static_cast<double>(ri) * static_cast<double>(ri);
        }
        if constexpr (X32) xi = static_cast<double>(static_cast<float>(xi));
        x[i] = xi;
    }
    block_sum_store<2>(acc, partials + (long)blockIdx.x * kPartialCols);
}

static int elementwise_blocks(long n)
{
    long nb = (n + kWG * 4 - 1) / (kWG * 4);
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    return (int)nb;
}

// The vector update streams six vectors in and two out: with up to 32768 workgroups (about ten
// 16-byte vectors per thread at 2560x1920x70) it moves 5.40 TB/s against 5.03 TB/s with 8192;
// its partial rows cost the single-workgroup sum 23 instead of 12 us.
static int update_blocks(long n)
{
    long nb = (n + kWG * 4 - 1) / (kWG * 4);
    if (nb > kUpdateMaxBlocks) nb = kUpdateMaxBlocks;
    if (nb < 1) nb = 1;
    return (int)nb;
}

void launch_update_mp(long n, double *x, const float *ph, const float *sh, const float *s, const float *t, float *r,
                      const float *rhat, double *partials, int *nrows, const Scalars *sc, bool x32, hipStream_t stream)
{
    const int nb = update_blocks(n);
    if (x32)
        hipLaunchKernelGGL(k_update_mp<true>, dim3(nb), dim3(kWG), 0, stream, n, x, ph, sh, s, t, r, rhat, partials, sc);
    else
        hipLaunchKernelGGL(k_update_mp<false>, dim3(nb), dim3(kWG), 0, stream, n, x, ph, sh, s, t, r, rhat, partials, sc);
    if (nrows) *nrows = nb;
}

template <typename Tv>
void launch_update(long n, Tv *x, const Tv *ph, const Tv *sh, const Tv *s, const Tv *t, Tv *r, const Tv *rhat,
                   double *partials, int *nrows, const Scalars *sc, hipStream_t stream)
{
    const int nb = update_blocks(n);
    hipLaunchKernelGGL((k_update<Tv>), dim3(nb), dim3(kWG), 0, stream, n, x, ph, sh, s, t, r, rhat, partials, sc);
    if (nrows) *nrows = nb;
}

// ------------------------------------------------------------------------------------------
// generic dot product (products and sums in FP64)
// ------------------------------------------------------------------------------------------
template <typename Ta, typename Tb>
__global__ __launch_bounds__(kWG) void k_dot(long n, const Ta *__restrict__ a, const Tb *__restrict__ b,
                                             double *__restrict__ partials)
{
    double acc[1] = {0.0};
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride)
        acc[0] += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    block_sum_store<1>(acc, partials + (long)blockIdx.x * kPartialCols);
}

template <typename Ta, typename Tb>
void launch_dot(long n, const Ta *a, const Tb *b, double *partials, int *nrows, hipStream_t s)
{
    const int nb = elementwise_blocks(n);
    hipLaunchKernelGGL((k_dot<Ta, Tb>), dim3(nb), dim3(kWG), 0, s, n, a, b, partials);
    if (nrows) *nrows = nb;
}

template <typename T>
__global__ __launch_bounds__(kWG) void k_dot2(long n, const T *__restrict__ a, const T *__restrict__ b,
                                              const T *__restrict__ c, const T *__restrict__ d,
                                              double *__restrict__ partials, const Scalars *__restrict__ sc,
                                              int stop_mask)
{
    if (stopped(sc, stop_mask)) return;
    double acc[2] = {0.0, 0.0};
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        acc[0] += static_cast<double>(a[i]) * static_cast<double>(b[i]);
        acc[1] += static_cast<double>(c[i]) * static_cast<double>(d[i]);
    }
    block_sum_store<2>(acc, partials + (long)blockIdx.x * kPartialCols);
}

template <typename T>
void launch_dot2(long n, const T *a, const T *b, const T *c, const T *d, double *partials, int *nrows,
                 const Scalars *sc, int stop_mask, hipStream_t s)
{
    const int nb = elementwise_blocks(n);
    hipLaunchKernelGGL((k_dot2<T>), dim3(nb), dim3(kWG), 0, s, n, a, b, c, d, partials, sc, stop_mask);
    if (nrows) *nrows = nb;
}

// ------------------------------------------------------------------------------------------
// Blocked Gram-Schmidt pieces for FGMRES: up to kMBlk basis vectors per pass (the basis is
// one array, vector i at V + i * n).
//   k_mdot   partials of <w, v_{i0+c}>, c < nb          (kMBlk columns per workgroup row)
//   k_maxpy  w -= sum_c h[i0+c] v_{i0+c} (sign -1) or x += sum_c h[i0+c] v_{i0+c} (sign +1);
//            with want_norm the partial of ||w||^2 after the update goes to column 0
// ------------------------------------------------------------------------------------------
template <typename Tv>
__global__ __launch_bounds__(kWG) void k_mdot(long n, const Tv *__restrict__ w, const Tv *__restrict__ V, int i0,
                                              int nb, double *__restrict__ part)
{
    double acc[kMBlk];
#pragma unroll
    for (int c = 0; c < kMBlk; ++c) acc[c] = 0.0;
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        const double wi = static_cast<double>(w[i]);
#pragma unroll
        for (int c = 0; c < kMBlk; ++c)
            if (c < nb) acc[c] += wi * static_cast<double>(V[(size_t)(i0 + c) * n + i]);
    }
    // fixed-order workgroup sum, kMBlk columns
    __shared__ double sm[kWG / 64][kMBlk];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < kMBlk; ++c) acc[c] += __shfl_xor(acc[c], off);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < kMBlk; ++c) sm[wv][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < kMBlk) {
        double s = sm[0][threadIdx.x];
        for (int w2 = 1; w2 < kWG / 64; ++w2) s += sm[w2][threadIdx.x];
        part[(long)blockIdx.x * kMBlk + threadIdx.x] = s;
    }
}

template <typename Tv>
__global__ __launch_bounds__(kWG) void k_maxpy(long n, Tv *__restrict__ w, const Tv *__restrict__ V, int i0, int nb,
                                               const double *__restrict__ h, double sign, int want_norm,
                                               double *__restrict__ part)
{
    Tv hc[kMBlk];
#pragma unroll
    for (int c = 0; c < kMBlk; ++c) hc[c] = (c < nb) ? static_cast<Tv>(sign * h[i0 + c]) : Tv(0);
    double acc[1] = {0.0};
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) {
        Tv wi = w[i];
#pragma unroll
        for (int c = 0; c < kMBlk; ++c)
            if (c < nb) wi += hc[c] * V[(size_t)(i0 + c) * n + i];
        w[i] = wi;
        acc[0] += static_cast<double>(wi) * static_cast<double>(wi);
    }
    if (want_norm) block_sum_store<1>(acc, part + (long)blockIdx.x * kPartialCols);
}

// out[c] = sum over rows of part[row][c], c < ncols (one workgroup; thread t sums the rows
// r = t / kMBlk (mod kWG / kMBlk) of column t % kMBlk, then the groups are added in order)
__global__ __launch_bounds__(kWG) void k_msum(const double *__restrict__ part, int rows, int ncols,
                                              double *__restrict__ out)
{
    constexpr int kGroups = kWG / kMBlk;
    __shared__ double sm[kWG];
    const int c = threadIdx.x % kMBlk, g = threadIdx.x / kMBlk;
    double s = 0.0;
    if (c < ncols) {
        // rows g, g + kGroups, ... added in that order, loaded eight at a time ahead
        constexpr int U = 8;
        int r = g;
        for (; r + (U - 1) * kGroups < rows; r += U * kGroups) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = part[(long)(r + u * kGroups) * kMBlk + c];
#pragma unroll
            for (int u = 0; u < U; ++u) s += v[u];
        }
        for (; r < rows; r += kGroups) s += part[(long)r * kMBlk + c];
    }
    sm[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < ncols) {
        double t = 0.0;
        for (int q = 0; q < kGroups; ++q) t += sm[q * kMBlk + threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// y = x * (1 / d[0])  (normalise the next Arnoldi vector by a device scalar)
template <typename Tv>
__global__ __launch_bounds__(kWG) void k_vscale(long n, const Tv *__restrict__ x, Tv *__restrict__ y,
                                                const double *__restrict__ d)
{
    const Tv s = static_cast<Tv>(1.0 / d[0]);
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) y[i] = x[i] * s;
}

template <typename Tv>
int launch_mdot(long n, const Tv *w, const Tv *V, int i0, int nb, double *part, double *out, hipStream_t s)
{
    // at most 2048 partial rows (8 workgroups per CU): enough to stream at full rate, few
    // enough for the single-workgroup column sums that follow
    const int rows = std::min(elementwise_blocks(n), 2048);
    hipLaunchKernelGGL((k_mdot<Tv>), dim3(rows), dim3(kWG), 0, s, n, w, V, i0, nb, part);
    hipLaunchKernelGGL(k_msum, dim3(1), dim3(kWG), 0, s, part, rows, nb, out + i0);
    return rows;
}

template <typename Tv>
int launch_maxpy(long n, Tv *w, const Tv *V, int i0, int nb, const double *h, double sign, int want_norm,
                 double *part, hipStream_t s)
{
    const int rows = elementwise_blocks(n);
    hipLaunchKernelGGL((k_maxpy<Tv>), dim3(rows), dim3(kWG), 0, s, n, w, V, i0, nb, h, sign, want_norm, part);
    return rows;
}

template <typename Tv> void launch_vscale(long n, const Tv *x, Tv *y, const double *d, hipStream_t s)
{
    hipLaunchKernelGGL((k_vscale<Tv>), dim3(elementwise_blocks(n)), dim3(kWG), 0, s, n, x, y, d);
}

// ------------------------------------------------------------------------------------------
// k_finalize: one workgroup.  Fixed-order FP64 reduction of the partial rows, then the
// scalar part of the iteration (thread 0).
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_finalize(int stage, const double *__restrict__ partials, int nrows,
                                                  Scalars *__restrict__ sc, double *__restrict__ hist,
                                                  double *__restrict__ out, int c_rr, int c_nb)
{
    double a[kPartialCols];
#pragma unroll
    for (int c = 0; c < kPartialCols; ++c) a[c] = 0.0;
    // thread t adds rows t, t + kWG, t + 2 kWG, ... in that order; the rows are loaded eight
    // at a time ahead of the additions (tens of thousands of rows on large grids: one load chain
    // per row would leave the single workgroup waiting on memory latency)
    constexpr int U = 8;
    int r = threadIdx.x;
    for (; r + (U - 1) * kWG < nrows; r += U * kWG) {
        double v[U][kPartialCols];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < kPartialCols; ++c) v[u][c] = partials[(long)(r + u * kWG) * kPartialCols + c];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int c = 0; c < kPartialCols; ++c) a[c] += v[u][c];
    }
    for (; r < nrows; r += kWG)
#pragma unroll
        for (int c = 0; c < kPartialCols; ++c) a[c] += partials[(long)r * kPartialCols + c];
    __shared__ double tot[kPartialCols];
    block_sum_store<kPartialCols>(a, tot);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double s0 = tot[0], s1 = tot[1], s2 = tot[2], s3 = tot[3];

    switch (stage) {
    case FIN_SUM:
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
        out[3] = s3;
        return;
    case FIN_INIT: {
        // start of a Krylov run: r = b - A x0 has just been formed
        const double nb2 = tot[c_nb], rr = tot[c_rr];
        sc->nb2 = nb2;
        sc->thr2 = sc->aux0 * sc->aux0 * nb2;   // aux0 carries tol
        sc->rr = rr;
        sc->iter = 0;
        sc->status = 0;
        sc->skip = sc->half = sc->wbd = 0;
        sc->restarts = 0;
        sc->fresh = 1;
        sc->was_fresh = 0;
        sc->rho = rr;
        sc->rhat2 = rr;
        sc->rho_prev = sc->alpha = sc->omega = 1.0;
        sc->beta = 0.0;
        sc->last_rel = nb2 > 0.0 ? sqrt(rr / nb2) : 0.0;
        sc->done = (nb2 == 0.0 || rr <= sc->thr2) ? 1 : 0;
        if (out) {
            out[0] = s0;
            out[1] = s1;
            out[2] = s2;
            out[3] = s3;
        }
        return;
    }
    case FIN_NET:
        // norms of the learned preconditioner's input and of its tridiagonal solve
        sc->net_q2 = s0;
        sc->net_z2 = s1;
        return;
    case FIN_LOSS:
        // training loss ||m - e||^2 / ||e||^2 of one pair, kept for the gradient seed
        sc->net_ee = s1;
        if (out) out[0] = s1 > 0.0 ? s0 / s1 : 0.0;
        return;
    case FIN_TRUE:
        // restart from a freshly computed true residual (periodic or residual-gap restart)
        sc->rr = tot[c_rr];
        sc->status = 0;
        sc->skip = sc->half = sc->wbd = 0;
        sc->fresh = 1;
        sc->rho = sc->rr;
        sc->rhat2 = sc->rr;
        sc->last_rel = sqrt(sc->rr / sc->nb2);
        sc->done = (sc->rr <= sc->thr2) ? 1 : 0;
        sc->restarts += 1;
        return;
    default:
        break;
    }
    if (sc->done) return;
    switch (stage) {
    case FIN_SIGMA: {
        const int wf = sc->fresh;
        sc->was_fresh = wf;
        sc->fresh = 0;
        const double sigma = s0, vv = s1;
        sc->work_mask = 0x3;   // thomas(P) and spmv(v) ran; the rest only if alpha is set
        if (!isfinite(sigma) || !isfinite(vv)) {   // poisoned iteration: stop
            sc->done = 1;
            sc->status = 2;
            sc->iter += 1;
            return;
        }
        if (fabs(sigma) <= sc->eps_bd * sqrt(sc->rhat2 * vv)) {
            if (wf) {               // breakdown right after a restart: nothing left to try
                sc->done = 1;
                sc->status = 2;
                sc->iter += 1;
                return;
            }
            sc->skip = 1;
            sc->restarts += 1;
            return;
        }
        sc->alpha = sc->rho / sigma;
        return;
    }
    case FIN_S:
        if (sc->skip) return;
        sc->ss = s0;
        if (s0 <= sc->thr2) sc->half = 1;
        return;
    case FIN_OMEGA:
        if (sc->skip || sc->half) return;
        if (s1 == 0.0 || s0 == 0.0) {
            sc->wbd = 1;
            sc->restarts += 1;
        } else {
            sc->omega = s0 / s1;
        }
        return;
    case FIN_END: {
        const int it = sc->iter + 1;
        sc->iter = it;
        const int slot = sc->hist_base + it - 1;
        sc->work_mask = sc->skip ? 0x3 : (sc->half ? 0x17 : 0x1f);
        if (sc->skip) {
            // sigma breakdown: r is unchanged, the next iteration starts afresh from it
            // (rhat = p = r), so the recurrence restarts from rho = ||r||^2 as after FIN_TRUE
            sc->skip = 0;
            sc->fresh = 1;
            sc->rho = sc->rr;
            sc->rhat2 = sc->rr;
            sc->rho_prev = sc->alpha = sc->omega = 1.0;
            sc->beta = 0.0;
            if (hist && slot < sc->hist_cap) hist[slot] = sc->last_rel;
            if (it >= sc->maxit) {
                sc->done = 1;
                sc->status = 1;
            }
            return;
        }
        if (sc->half) {
            sc->last_rel = sqrt(sc->ss / sc->nb2);
            if (hist && slot < sc->hist_cap) hist[slot] = sc->last_rel;
            sc->done = 1;
            sc->status = 0;
            return;
        }
        const double rr = s1;
        sc->rr = rr;
        sc->last_rel = sqrt(rr / sc->nb2);
        if (hist && slot < sc->hist_cap) hist[slot] = sc->last_rel;
        if (!isfinite(rr) || !isfinite(s0)) {
            sc->done = 1;
            sc->status = 2;
            return;
        }
        if (sc->wbd) {
            sc->wbd = 0;
            sc->fresh = 1;
        }
        if (rr <= sc->thr2) {
            sc->done = 1;
            sc->status = 0;
            return;
        }
        if (it >= sc->maxit) {
            sc->done = 1;
            sc->status = 1;
            return;
        }
        if (sc->restart_every > 0 && it % sc->restart_every == 0) {
            sc->done = 1;
            sc->status = 4;
            return;
        }
        if (sc->fresh) {
            sc->rho = rr;
            sc->rhat2 = rr;
            sc->rho_prev = sc->alpha = sc->omega = 1.0;
            sc->beta = 0.0;
            return;
        }
        const double rhr = s0;
        if (fabs(rhr) <= sc->eps_bd * sqrt(sc->rhat2 * rr)) {
            sc->fresh = 1;
            sc->restarts += 1;
            sc->rho = rr;
            sc->rhat2 = rr;
            sc->rho_prev = sc->alpha = sc->omega = 1.0;
            sc->beta = 0.0;
            return;
        }
        sc->rho_prev = sc->rho;
        sc->beta = (rhr / sc->rho) * (sc->alpha / sc->omega);
        sc->rho = rhr;
        return;
    }
    default:
        return;
    }
}

void launch_finalize(int stage, const double *partials, int nrows, Scalars *sc, double *hist, double *out,
                     int c_rr, int c_nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kWG), 0, s, stage, partials, nrows, sc, hist, out, c_rr, c_nb);
}

// ------------------------------------------------------------------------------------------
// small elementwise kernels
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWG) void k_fill(T *p, long n, T v)
{
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T> void launch_fill(T *p, long n, T v, hipStream_t s)
{
    hipLaunchKernelGGL((k_fill<T>), dim3(elementwise_blocks(n)), dim3(kWG), 0, s, p, n, v);
}

// x64 += d32 (the FP64 solution update of a refinement step)
__global__ __launch_bounds__(kWG) void k_add_correction(long n, double *__restrict__ x, const float *__restrict__ d)
{
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) x[i] += static_cast<double>(d[i]);
}

void launch_add_correction(long n, double *x, const float *d, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_correction, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, n, x, d);
}

// out = float(a - b)   (harvest: error of an iterate against the reference solution)
__global__ __launch_bounds__(kWG) void k_sub_to_f32(long n, const double *__restrict__ a, const double *__restrict__ b,
                                                    float *__restrict__ out)
{
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) out[i] = static_cast<float>(a[i] - b[i]);
}

void launch_sub_to_f32(long n, const double *a, const double *b, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_to_f32, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, n, a, b, out);
}

__global__ __launch_bounds__(kWG) void k_cast_f32(long n, const double *__restrict__ a, float *__restrict__ out)
{
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride) out[i] = static_cast<float>(a[i]);
}

void launch_cast_f32(long n, const double *a, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast_f32, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, n, a, out);
}

__global__ __launch_bounds__(kWG) void k_check_finite(long n, const double *__restrict__ v, int *bad)
{
    int cnt = 0;
    const long stride = (long)gridDim.x * kWG;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += stride)
        if (!isfinite(v[i])) ++cnt;
    if (cnt) atomicAdd(bad, cnt);
}

void launch_check_finite(long n, const double *v, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_finite, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, n, v, bad);
}

// ------------------------------------------------------------------------------------------
// operator setup
// ------------------------------------------------------------------------------------------
// Copy the couplings, derive the margin m = C - (((((W+E)+S)+N)+D)+U), and count violations: bad[0] non-finite, bad[1] negative coupling, bad[2] coupling across a
// pole / the bottom / the top, bad[3] non-positive margin.
__global__ __launch_bounds__(kWG) void k_derive(const double *__restrict__ cf, int nlon, int nlat, int nlev,
                                                double *__restrict__ a64, double *__restrict__ m64,
                                                int *__restrict__ bad)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    int b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    const long stride = (long)gridDim.x * kWG;
    for (long c = (long)blockIdx.x * kWG + threadIdx.x; c < n; c += stride) {
        const int j = (int)((c / nlon) % nlat);
        const int k = (int)(c / P);
        double a[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            a[d] = cf[d * n + c];
            a64[d * n + c] = a[d];
            if (!isfinite(a[d])) ++b0;
            else if (a[d] < 0.0) ++b1;
        }
        const double C = cf[6 * n + c];
        if (!isfinite(C)) ++b0;
        if ((j == 0 && a[2] != 0.0) || (j == nlat - 1 && a[3] != 0.0) || (k == 0 && a[4] != 0.0) ||
            (k == nlev - 1 && a[5] != 0.0))
            ++b2;
        const double hs = ((a[0] + a[1]) + a[2]) + a[3];
        const double m = C - ((hs + a[4]) + a[5]);
        if (!(m > 0.0)) ++b3;
        m64[c] = m;
    }
    if (b0) atomicAdd(bad + 0, b0);
    if (b1) atomicAdd(bad + 1, b1);
    if (b2) atomicAdd(bad + 2, b2);
    if (b3) atomicAdd(bad + 3, b3);
}

void launch_derive(const double *coeffs, int nlon, int nlat, int nlev, double *a64, double *m64, int *bad,
                   hipStream_t s)
{
    const long n = (long)nlon * nlat * nlev;
    hipLaunchKernelGGL(k_derive, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, coeffs, nlon, nlat, nlev, a64, m64,
                       bad);
}

__global__ __launch_bounds__(kWG) void k_to_fp32(long n, const double *__restrict__ a64,
                                                 const double *__restrict__ m64, float *__restrict__ a32,
                                                 float *__restrict__ m32)
{
    const long stride = (long)gridDim.x * kWG;
    for (long c = (long)blockIdx.x * kWG + threadIdx.x; c < n; c += stride) {
#pragma unroll
        for (int d = 0; d < 6; ++d) a32[d * n + c] = static_cast<float>(a64[d * n + c]);
        m32[c] = static_cast<float>(m64[c]);
    }
}

void launch_to_fp32(long n, const double *a64, const double *m64, float *a32, float *m32, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_fp32, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, n, a64, m64, a32, m32);
}

// Round a double to p significant bits, ties to even, with exponents below emin held at emin
// (gradual underflow); the sign is kept.  Every step is exact except the single rint.
__device__ double round_sig(double u, int p, int emin)
{
    if (u == 0.0) return 0.0;
    int e;
    (void)frexp(u, &e);         // |u| = f 2^e, f in [1/2, 1): leading bit has weight 2^(e-1)
    int lead = e - 1;
    if (lead < emin) lead = emin;
    const double ulp = ldexp(1.0, lead - (p - 1));
    return rint(u / ulp) * ulp;
}

// One wave per (direction, level, latitude row).  Offset: the FP32 rounding of the midpoint of
// the row's smallest and largest coupling when every coupling of the row is positive and the
// largest is at most twice the smallest, else 0 (zero couplings stay zero, and no coupling's
// relative error exceeds the plain format's); scale: the power of two 2^ceil(log2 max
// |a - offset|).  Stored at qs[(k * nlat + j) * kQsStride + d] and + kQsOff + d, so one row's
// record is one 64-byte line.
__global__ __launch_bounds__(64) void k_qscale(int nlon, int nlat, int nlev, const double *__restrict__ a64,
                                               float *__restrict__ qs)
{
    const long row = blockIdx.x;   // (d * nlev + k) * nlat + j
    const int d = (int)(row / ((long)nlev * nlat));
    const long kj = row % ((long)nlev * nlat);
    const long n = (long)nlon * nlat * nlev;
    const double *src = a64 + (long)d * n + kj * nlon;
    double lo = INFINITY, hi = 0.0;
    for (int i = threadIdx.x; i < nlon; i += 64) {
        lo = fmin(lo, src[i]);
        hi = fmax(hi, src[i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    const float offv = (lo > 0.0 && hi <= 2.0 * lo) ? static_cast<float>(0.5 * (lo + hi)) : 0.f;
    double mx = 0.0;
    for (int i = threadIdx.x; i < nlon; i += 64) mx = fmax(mx, fabs(src[i] - static_cast<double>(offv)));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (threadIdx.x == 0) {
        float s = 1.f;
        if (mx > 0.0) {
            int e;
            const double f = frexp(mx, &e);
            s = ldexpf(1.f, (f == 0.5) ? e - 1 : e);
        }
        qs[kj * kQsStride + d] = s;
        qs[kj * kQsStride + kQsOff + d] = offv;
        if (d == 0)
            for (int pad = 6; pad < kQsOff; ++pad) {
                qs[kj * kQsStride + pad] = 1.f;
                qs[kj * kQsStride + kQsOff + pad] = 0.f;
            }
    }
}

// q = RNE((a - offset) / scale) in BF16 (kind 2) or FP16 (kind 3)
__global__ __launch_bounds__(kWG) void k_quantize(int kind, int nlon, int nlat, int nlev,
                                                  const double *__restrict__ a64, const float *__restrict__ qs,
                                                  uint16_t *__restrict__ aq)
{
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    const long stride = (long)gridDim.x * kWG;
    for (long c = (long)blockIdx.x * kWG + threadIdx.x; c < n; c += stride) {
        const long kj = c / nlon;   // k * nlat + j
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const double s = qs[kj * kQsStride + d];
            const double off = qs[kj * kQsStride + kQsOff + d];
            const double u = (a64[d * n + c] - off) / s;
            uint16_t bits;
            if (kind == PBF16) {
                const double r = round_sig(u, 8, -126);
                bits = static_cast<uint16_t>(__float_as_uint(static_cast<float>(r)) >> 16);
            } else {
                const double r = round_sig(u, 11, -14);
                const _Float16 h = static_cast<_Float16>(static_cast<float>(r));
                bits = __builtin_bit_cast(uint16_t, h);
            }
            aq[d * n + c] = bits;
        }
    }
}

void launch_quantize(int kind, int nlon, int nlat, int nlev, const double *a64, uint16_t *aq, float *qs,
                     hipStream_t s)
{
    const long rows = 6L * nlev * nlat;
    hipLaunchKernelGGL(k_qscale, dim3((unsigned)rows), dim3(64), 0, s, nlon, nlat, nlev, a64, qs);
    const long n = (long)nlon * nlat * nlev;
    hipLaunchKernelGGL(k_quantize, dim3(elementwise_blocks(n)), dim3(kWG), 0, s, kind, nlon, nlat, nlev, a64, qs,
                       aq);
}

// ------------------------------------------------------------------------------------------
// Red-black vertical-line SOR (Sec. 2, Eq. 6-7, the tri_sor preconditioner with the columns
// visited in red-black order; red: i + j even).  A sweep updates every column of one colour,
// then every column of the other, each by
//     x_c <- (1 - omega) x_c + omega T_c^{-1} (q_c + sum of its horizontal couplings times x)
// With nlon even every horizontal neighbour has the other colour, so the columns of one colour
// are independent: one lane per column, the rhs gathered level by level on the way up, w_k of
// the Thomas forward sweep kept (in registers at 70 levels, k_sor_half_reg; otherwise parked
// in a scratch vector, k_sor_half), the blend done on the way down.
//
// Layout: everything a half-sweep touches is in colour-major order,
// index = colour * n/2 + k * P/2 + c2 with c2 = j * nlon/2 + i/2: the operator constants (the
// three LU factors of T and the W, E, S, N couplings, a second copy made once), q and x.  The
// lanes of a wave hold 64 consecutive columns of one colour in a latitude row, so every access
// is unit-stride: own constants, q and x at c2, the other colour's west/east neighbours at
// c2 - 1 + par and c2 + par (par = parity of i; with the periodic wrap in longitude) and its
// south/north neighbours at c2 -/+ nlon/2.  The tridiagonal kernel writes T^{-1} q and q in this
// order (k_thomas with CM); the last half-sweep writes the result in grid order, each lane the
// pair of grid columns 2m, 2m + 1 of its row (its own column and the other colour's partner).
//
// The first half-sweep from x = 0 is omega T^{-1} q on the red columns; the tridiagonal kernel
// has already computed T^{-1} q for every column, so the chain starts at the first black
// half-sweep and reads the red values with the factor omega applied on the fly (nb_scale),
// and the next red half-sweep reads its own old value the same way (own_scale).
// ------------------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWG) void k_sor_perm(const T *__restrict__ src, T *__restrict__ dst, int nd, int nlon,
                                                  int nlat, int nlev)
{
    const long P = (long)nlon * nlat, n = P * nlev, P2 = P / 2;
    const long total = (long)nd * n;
    const long stride = (long)gridDim.x * kWG;
    for (long e = (long)blockIdx.x * kWG + threadIdx.x; e < total; e += stride) {
        const long d = e / n, c = e % n;
        const long k = c / P, pc = c % P;
        const int j = (int)(pc / nlon), i = (int)(pc % nlon);
        const int colour = (i + j) & 1;
        const long c2 = (long)j * (nlon / 2) + i / 2;
        dst[d * n + colour * (n / 2) + k * P2 + c2] = src[e];
    }
}

// One wave per workgroup for the half-sweeps too (133-233 VGPRs: a finished wave is replaced on
// its own SIMD at once).
constexpr int kSorWG = 64;

template <typename Tv, typename Tc, bool LAST>
__global__ __launch_bounds__(kSorWG) void k_sor_half(OpView<Tc> op, SorView<Tv, Tc> sv, const Tv *__restrict__ qcm,
                                                  Tv *__restrict__ xcm, Tv *__restrict__ wsc, Tv *__restrict__ xout,
                                                  int colour, Tv omega, Tv nb_scale, Tv own_scale,
                                                  const Scalars *__restrict__ sc, int stop_mask, int per_xcd)
{
    if (stopped(sc, stop_mask)) return;
    using V = typename CoefTraits<Tc>::val;
    constexpr bool Q = CoefTraits<Tc>::quant;
    const int nlat = op.nlat, nlev = op.nlev;
    const int half = op.nlon / 2;
    const long P = op.P, n = op.n, P2 = P / 2, n2 = n / 2;
    // XCD-aware: workgroups go round-robin over the 8 XCDs, so workgroup b takes the logical
    // block (b % 8) * per_xcd + b / 8 and each XCD walks a contiguous band of latitude rows,
    // whose north and south neighbour rows its own L2 then holds
    const long lb = (long)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const long c2 = lb * kSorWG + threadIdx.x;
    if (c2 >= P2) return;
    const int j = (int)(c2 / half), m = (int)(c2 % half);
    const int par = (j + colour) & 1;   // own grid column i = 2m + par
    // the other colour's west / east neighbours in this row (periodic in longitude)
    const long cw = (long)j * half + (par ? m : (m == 0 ? half - 1 : m - 1));
    const long ce = (long)j * half + (par ? (m == half - 1 ? 0 : m + 1) : m);
    const long own = (long)colour * n2 + c2;
    const Tv *oth = xcm + (long)(1 - colour) * n2;
    const bool hs = j > 0, hn = j < nlat - 1;
    const Tv *lf = sv.f, *invf = sv.f + n, *cf = sv.f + 2 * n;
    const Tc *aWp = sv.a, *aEp = sv.a + n, *aSp = sv.a + 2 * n, *aNp = sv.a + 3 * n;
    Tv wprev = 0;
    for (int k = 0; k < nlev; ++k) {
        const long pi = own + (long)k * P2;
        const Tv *ok = oth + (long)k * P2;
        float s0 = 1.f, s1 = 1.f, s2 = 1.f, s3 = 1.f, f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
        if constexpr (Q) {
            const float *qr = op.qs + ((size_t)k * nlat + j) * kQsStride;
            s0 = qr[0];
            s1 = qr[1];
            s2 = qr[2];
            s3 = qr[3];
            f0 = qr[kQsOff];
            f1 = qr[kQsOff + 1];
            f2 = qr[kQsOff + 2];
            f3 = qr[kQsOff + 3];
        }
        const V aW = DecB<Tc>::get(aWp + pi, 0, s0, f0);
        const V aE = DecB<Tc>::get(aEp + pi, 0, s1, f1);
        Tv h = aW * ok[cw] + aE * ok[ce];
        if (hs) h += static_cast<Tv>(DecB<Tc>::get(aSp + pi, 0, s2, f2)) * ok[c2 - half];
        if (hn) h += static_cast<Tv>(DecB<Tc>::get(aNp + pi, 0, s3, f3)) * ok[c2 + half];
        const Tv rhs = __builtin_nontemporal_load(qcm + pi) + nb_scale * h;
        const Tv w = rhs + __builtin_nontemporal_load(lf + pi) * wprev;
        __builtin_nontemporal_store(w, wsc + c2 + (long)k * P2);
        wprev = w;
    }
    const Tv keep = (Tv(1) - omega) * own_scale;
    Tv ynext = 0;
    for (int k = nlev - 1; k >= 0; --k) {
        const long pi = own + (long)k * P2;
        const Tv y = __builtin_nontemporal_load(invf + pi) * __builtin_nontemporal_load(wsc + c2 + (long)k * P2) +
                     __builtin_nontemporal_load(cf + pi) * ynext;
        const Tv old = (own_scale == Tv(0)) ? Tv(0) : xcm[pi];
        const Tv val = keep * old + omega * y;
        if constexpr (LAST) {
            // grid columns 2m and 2m + 1 of row j: this column (2m + par) and its partner of
            // the other colour, which has the same c2; the wave writes whole cache lines
            Tv *o = xout + (long)k * P + 2 * c2;
            __builtin_nontemporal_store(val, o + par);
            __builtin_nontemporal_store(nb_scale * oth[(long)k * P2 + c2], o + (1 - par));
        } else {
            xcm[pi] = val;
        }
        ynext = y;
    }
}

// Register-resident variant for a fixed level count NL: the forward values w_k stay in
// registers (no parked vector: 4 B per point less per FP32 half-sweep).  The loads of level
// k + PF are issued while level k is computed, into a ring of PF register slots, with
// scheduling fences so the compiler does not hoist every level's loads (as in k_thomas).
// Needs nlon/2 % 64 == 0, so that each wave lies within one latitude row; the south/north
// loads of the first/last row read the own column instead (their couplings are zero there, so
// the sum is the same as the generic kernel's, which skips them).
template <typename Tv, typename Tc, bool LAST, int NL, int PF>
__device__ __forceinline__ void sor_half_reg_body(OpView<Tc> op, SorView<Tv, Tc> sv, const Tv *__restrict__ qcm,
                                                  Tv *__restrict__ xcm, Tv *__restrict__ xout, int colour, Tv omega,
                                                  Tv nb_scale, Tv own_scale, const Scalars *__restrict__ sc,
                                                  int stop_mask, int per_xcd)
{
    if (stopped(sc, stop_mask)) return;
    using V = typename CoefTraits<Tc>::val;
    constexpr bool Q = CoefTraits<Tc>::quant;
    const int nlat = op.nlat;
    const int half = op.nlon / 2;
    const long P = op.P, n = op.n, P2 = P / 2, n2 = n / 2;
    const long lb = (long)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const long c2 = lb * kSorWG + threadIdx.x;
    if (c2 >= P2) return;   // whole waves (P/2 is a multiple of 64 here)
    const int j = __builtin_amdgcn_readfirstlane((int)(c2 / half));
    const int m = (int)(c2 - (long)j * half);
    const int par = (j + colour) & 1;
    constexpr uint32_t SV = sizeof(Tv);
    // lane byte offsets within a level plane of one colour
    const uint32_t oo = (uint32_t)c2 * SV;
    const uint32_t ow = (uint32_t)(j * half + (par ? m : (m == 0 ? half - 1 : m - 1))) * SV;
    const uint32_t oe = (uint32_t)(j * half + (par ? (m == half - 1 ? 0 : m + 1) : m)) * SV;
    const uint32_t os = (j > 0) ? oo - (uint32_t)half * SV : oo;
    const uint32_t on = (j < nlat - 1) ? oo + (uint32_t)half * SV : oo;
    const uint32_t oc = (uint32_t)c2;   // element index into the coupling rows
    const Tv *qb = qcm + (long)colour * n2;
    const Tv *lfb = sv.f + (long)colour * n2, *invb = sv.f + n + (long)colour * n2, *cfb = sv.f + 2 * n + (long)colour * n2;
    const Tc *aWb = sv.a + (long)colour * n2, *aEb = aWb + n, *aSb = aWb + 2 * n, *aNb = aWb + 3 * n;
    const Tv *oth = xcm + (long)(1 - colour) * n2;
    Tv *own = xcm + (long)colour * n2;

    Tv w[NL];
    {
        V rw[PF], re[PF], rs[PF], rn[PF];
        Tv xw[PF], xe[PF], xs[PF], xn[PF], rq[PF], rl[PF];
        auto issue = [&](int kk, int sl) {
            const size_t lo = (size_t)kk * (size_t)P2;
            float s0 = 1.f, s1 = 1.f, s2 = 1.f, s3 = 1.f, f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
            if constexpr (Q) {
                const float *rec = op.qs + ((size_t)kk * nlat + j) * kQsStride;
                const float4 sq = *reinterpret_cast<const float4 *>(rec);
                const float4 oq = *reinterpret_cast<const float4 *>(rec + kQsOff);
                s0 = sq.x;
                s1 = sq.y;
                s2 = sq.z;
                s3 = sq.w;
                f0 = oq.x;
                f1 = oq.y;
                f2 = oq.z;
                f3 = oq.w;
            }
            rw[sl] = DecB<Tc>::get(aWb + lo, oc, s0, f0);
            re[sl] = DecB<Tc>::get(aEb + lo, oc, s1, f1);
            rs[sl] = DecB<Tc>::get(aSb + lo, oc, s2, f2);
            rn[sl] = DecB<Tc>::get(aNb + lo, oc, s3, f3);
            xw[sl] = ldb(oth + lo, ow);
            xe[sl] = ldb(oth + lo, oe);
            xs[sl] = ldb(oth + lo, os);
            xn[sl] = ldb(oth + lo, on);
            rq[sl] = ldn(qb + lo, oo);
            rl[sl] = ldn(lfb + lo, oo);
        };
#pragma unroll
        for (int k = 0; k < PF && k < NL; ++k) issue(k, k);
        Tv wprev = 0;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int sl = k % PF;
            Tv h = rw[sl] * xw[sl] + re[sl] * xe[sl];
            h += static_cast<Tv>(rs[sl]) * xs[sl];
            h += static_cast<Tv>(rn[sl]) * xn[sl];
            const Tv rhs = rq[sl] + nb_scale * h;
            w[k] = rhs + rl[sl] * wprev;
            wprev = w[k];
            if (k + PF < NL) issue(k + PF, sl);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    const Tv keep = (Tv(1) - omega) * own_scale;
    auto backward = [&](auto own_c) {
        constexpr bool OWN = decltype(own_c)::value;
        Tv bi[PF], bc[PF], bo[PF], bp[PF];
        auto issue = [&](int kk, int sl) {
            const size_t lo = (size_t)kk * (size_t)P2;
            bi[sl] = ldn(invb + lo, oo);
            bc[sl] = ldn(cfb + lo, oo);
            if constexpr (OWN) bo[sl] = ldb(own + lo, oo);
            if constexpr (LAST) bp[sl] = ldb(oth + lo, oo);
        };
#pragma unroll
        for (int t = 0; t < PF && t < NL; ++t) issue(NL - 1 - t, t);
        Tv ynext = 0;
#pragma unroll
        for (int k = NL - 1; k >= 0; --k) {
            const int sl = (NL - 1 - k) % PF;
            const Tv y = bi[sl] * w[k] + bc[sl] * ynext;
            const Tv old = OWN ? bo[sl] : Tv(0);
            const Tv val = keep * old + omega * y;
            if constexpr (LAST) {
                Tv *o = xout + (size_t)k * (size_t)P;
                const uint32_t g = (uint32_t)(2 * c2);
                __builtin_nontemporal_store(val, o + g + par);
                __builtin_nontemporal_store(nb_scale * bp[sl], o + g + (1 - par));
            } else {
                stb(own + (size_t)k * (size_t)P2, oo, val);
            }
            ynext = y;
            if (k - PF >= 0) issue(k - PF, sl);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (own_scale == Tv(0))
        backward(std::integral_constant<bool, false>{});
    else
        backward(std::integral_constant<bool, true>{});
}

template <typename Tv, typename Tc, bool LAST, int NL, int PF>
__global__ __launch_bounds__(kSorWG) void k_sor_half_reg(OpView<Tc> op, SorView<Tv, Tc> sv, const Tv *__restrict__ qcm,
                                                      Tv *__restrict__ xcm, Tv *__restrict__ xout, int colour,
                                                      Tv omega, Tv nb_scale, Tv own_scale,
                                                      const Scalars *__restrict__ sc, int stop_mask, int per_xcd)
{
    sor_half_reg_body<Tv, Tc, LAST, NL, PF>(op, sv, qcm, xcm, xout, colour, omega, nb_scale, own_scale, sc, stop_mask,
                                            per_xcd);
}

// 140 levels in FP64: one wave per SIMD with the whole register file, as k_thomas_deep
template <typename Tv, typename Tc, bool LAST, int NL, int PF>
__global__ __launch_bounds__(kSorWG) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_sor_half_deep(
    OpView<Tc> op, SorView<Tv, Tc> sv, const Tv *__restrict__ qcm, Tv *__restrict__ xcm, Tv *__restrict__ xout,
    int colour, Tv omega, Tv nb_scale, Tv own_scale, const Scalars *__restrict__ sc, int stop_mask, int per_xcd)
{
    sor_half_reg_body<Tv, Tc, LAST, NL, PF>(op, sv, qcm, xcm, xout, colour, omega, nb_scale, own_scale, sc, stop_mask,
                                            per_xcd);
}

template <typename T> void launch_sor_perm(const T *src, T *dst, int nd, int nlon, int nlat, int nlev, hipStream_t s)
{
    const long n = (long)nlon * nlat * nlev;
    hipLaunchKernelGGL((k_sor_perm<T>), dim3(elementwise_blocks(nd * n)), dim3(kWG), 0, s, src, dst, nd, nlon, nlat,
                       nlev);
}

// levels in flight in the register-resident half-sweep (FP32 and FP64 vectors: 138 and 233
// VGPRs, no spills)
constexpr int kSorPF = 4;
constexpr int kSorPF64 = 3;
constexpr int kSorDeepPF = 8;   // 140 levels in FP64, one wave per SIMD

template <typename Tv, typename Tc>
void launch_sor(const OpView<Tc> &op, const SorView<Tv, Tc> &sv, const Tv *qcm, Tv *xcm, Tv *wsc, Tv *xout,
                int sweeps, double omega, const Scalars *sc, int stop_mask, hipStream_t s)
{
    const long half_cols = op.P / 2;
    const long lblocks = (half_cols + kSorWG - 1) / kSorWG;
    const int per_xcd = (int)((lblocks + 7) / 8);
    const unsigned blocks = (unsigned)(per_xcd * 8);
    const Tv w = static_cast<Tv>(omega);
    const int last = 2 * sweeps - 1;
    // register-resident forward values at 70 and 140 levels, when each wave lies within one
    // latitude row and level offsets fit 32 bits
    const bool rows_ok = (op.nlon / 2) % 64 == 0 && (unsigned long)op.n * sizeof(Tv) < (1ul << 32);
    const bool reg = rows_ok && op.nlev == 70;
    const bool reg140 = rows_ok && op.nlev == 140;
    for (int h = 1; h <= last; ++h) {
        const int colour = (h & 1) ? 1 : 0;                       // odd: black, even: red
        const Tv nb_scale = (h == 1) ? w : Tv(1);                 // red still holds T^{-1} q
        const Tv own_scale = (h == 1) ? Tv(0) : (h == 2 ? w : Tv(1));
        if (reg) {
            constexpr int PF = sizeof(Tv) == 4 ? kSorPF : kSorPF64;
            if (h == last)
                hipLaunchKernelGGL((k_sor_half_reg<Tv, Tc, true, 70, PF>), dim3(blocks), dim3(kSorWG), 0, s, op, sv, qcm,
                                   xcm, xout, colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
            else
                hipLaunchKernelGGL((k_sor_half_reg<Tv, Tc, false, 70, PF>), dim3(blocks), dim3(kSorWG), 0, s, op, sv, qcm,
                                   xcm, xout, colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
            continue;
        }
        if (reg140) {
            if constexpr (sizeof(Tv) == 4) {
                if (h == last)
                    hipLaunchKernelGGL((k_sor_half_reg<Tv, Tc, true, 140, kSorPF>), dim3(blocks), dim3(kSorWG), 0, s, op,
                                       sv, qcm, xcm, xout, colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
                else
                    hipLaunchKernelGGL((k_sor_half_reg<Tv, Tc, false, 140, kSorPF>), dim3(blocks), dim3(kSorWG), 0, s,
                                       op, sv, qcm, xcm, xout, colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
            } else {
                if (h == last)
                    hipLaunchKernelGGL((k_sor_half_deep<Tv, Tc, true, 140, kSorDeepPF>), dim3(blocks), dim3(kSorWG), 0, s,
                                       op, sv, qcm, xcm, xout, colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
                else
                    hipLaunchKernelGGL((k_sor_half_deep<Tv, Tc, false, 140, kSorDeepPF>), dim3(blocks), dim3(kSorWG), 0,
                                       s, op, sv, qcm, xcm, xout, colour, w, nb_scale, own_scale, sc, stop_mask,
                                       per_xcd);
            }
            continue;
        }
        if (h == last)
            hipLaunchKernelGGL((k_sor_half<Tv, Tc, true>), dim3(blocks), dim3(kSorWG), 0, s, op, sv, qcm, xcm, wsc, xout,
                               colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
        else
            hipLaunchKernelGGL((k_sor_half<Tv, Tc, false>), dim3(blocks), dim3(kSorWG), 0, s, op, sv, qcm, xcm, wsc,
                               xout, colour, w, nb_scale, own_scale, sc, stop_mask, per_xcd);
    }
}

// ------------------------------------------------------------------------------------------
// explicit instantiations
// ------------------------------------------------------------------------------------------
template void launch_spmv<double, double>(const OpView<double> &, const double *, double *, const double *, int,
                                          double *, int *, const Scalars *, int, hipStream_t);
template void launch_spmv<float, float>(const OpView<float> &, const float *, float *, const float *, int, double *,
                                        int *, const Scalars *, int, hipStream_t);
template void launch_spmv<float, bf16_t>(const OpView<bf16_t> &, const float *, float *, const float *, int,
                                         double *, int *, const Scalars *, int, hipStream_t);
template void launch_spmv<float, fp16_t>(const OpView<fp16_t> &, const float *, float *, const float *, int,
                                         double *, int *, const Scalars *, int, hipStream_t);
template void launch_residual<double>(const OpView<double> &, const double *, const double *, double *, double *,
                                      int *, hipStream_t);
template void launch_residual<float>(const OpView<double> &, const double *, const double *, float *, double *,
                                     int *, hipStream_t);
template void launch_thomas<double>(const TriView<double> &, const double *, double *, int, const double *,
                                    double *, const double *, double *, double *, int *, const Scalars *, hipStream_t,
                                    int);
template void launch_thomas<float>(const TriView<float> &, const float *, float *, int, const float *, float *,
                                   const float *, float *, double *, int *, const Scalars *, hipStream_t, int);
template void launch_thomas_cm<double>(const TriView<double> &, int, const double *, double *, double *, int,
                                       const double *, double *, const double *, double *, double *, int *,
                                       const Scalars *, hipStream_t, int);
template void launch_thomas_cm<float>(const TriView<float> &, int, const float *, float *, float *, int,
                                      const float *, float *, const float *, float *, double *, int *,
                                      const Scalars *, hipStream_t, int);
template void launch_tri_factor<double>(const double *, const double *, int, int, int, double *, hipStream_t);
template void launch_tri_factor<float>(const double *, const double *, int, int, int, float *, hipStream_t);
template void launch_update<double>(long, double *, const double *, const double *, const double *, const double *,
                                    double *, const double *, double *, int *, const Scalars *, hipStream_t);
template void launch_update<float>(long, float *, const float *, const float *, const float *, const float *,
                                   float *, const float *, double *, int *, const Scalars *, hipStream_t);
template void launch_dot<double, double>(long, const double *, const double *, double *, int *, hipStream_t);
template void launch_dot<float, float>(long, const float *, const float *, double *, int *, hipStream_t);
template void launch_dot2<double>(long, const double *, const double *, const double *, const double *, double *,
                                  int *, const Scalars *, int, hipStream_t);
template void launch_dot2<float>(long, const float *, const float *, const float *, const float *, double *, int *,
                                 const Scalars *, int, hipStream_t);
template int launch_mdot<double>(long, const double *, const double *, int, int, double *, double *, hipStream_t);
template int launch_mdot<float>(long, const float *, const float *, int, int, double *, double *, hipStream_t);
template int launch_maxpy<double>(long, double *, const double *, int, int, const double *, double, int, double *,
                                  hipStream_t);
template int launch_maxpy<float>(long, float *, const float *, int, int, const double *, double, int, double *,
                                 hipStream_t);
template void launch_vscale<double>(long, const double *, double *, const double *, hipStream_t);
template void launch_vscale<float>(long, const float *, float *, const double *, hipStream_t);
template void launch_sor<double, double>(const OpView<double> &, const SorView<double, double> &, const double *,
                                         double *, double *, double *, int, double, const Scalars *, int, hipStream_t);
template void launch_sor<float, float>(const OpView<float> &, const SorView<float, float> &, const float *, float *,
                                       float *, float *, int, double, const Scalars *, int, hipStream_t);
template void launch_sor<float, bf16_t>(const OpView<bf16_t> &, const SorView<float, bf16_t> &, const float *,
                                        float *, float *, float *, int, double, const Scalars *, int, hipStream_t);
template void launch_sor<float, fp16_t>(const OpView<fp16_t> &, const SorView<float, fp16_t> &, const float *,
                                        float *, float *, float *, int, double, const Scalars *, int, hipStream_t);
template void launch_sor_perm<double>(const double *, double *, int, int, int, int, hipStream_t);
template void launch_sor_perm<float>(const float *, float *, int, int, int, int, hipStream_t);
template void launch_sor_perm<uint16_t>(const uint16_t *, uint16_t *, int, int, int, int, hipStream_t);
template void launch_fill<double>(double *, long, double, hipStream_t);
template void launch_fill<float>(float *, long, float, hipStream_t);

}  // namespace eg
