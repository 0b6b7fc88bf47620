// Internal declarations of the endgame library (not part of the public ABI).
//
// Storage of an operator on the device (one set per precision, struct-of-arrays, each array
// laid out like the grid, idx = i + nlon*(j + nlat*k)):
//   a[6][n]  couplings W, E, S, N, D, U (magnitudes; matrix entries are their negatives)
//   m[n]     margin  C - sum(a)  (> 0): the SpMV runs in the difference form
//            y = m x + sum_d a_d (x - x_d), which never forms C x - sum a_d x_d and so keeps
//            the small margin exact in FP32 and 16-bit storage
//   f[3][n]  LU factors (l, inv, c) of the vertical tridiagonal T, computed once in FP64
// 16-bit sets store a[] as BF16/FP16 bits scaled by a power of two per (direction, level,
// latitude row) and share m and the FP32 factors with the FP32 set.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace eg {

constexpr int kWG = 256;                 // threads per workgroup of the streaming kernels
constexpr int kPartialCols = 4;          // doubles per partial row

enum Prec { P64 = 0, P32 = 1, PBF16 = 2, PFP16 = 3 };

// Device-resident state of one Krylov run.  Written only by the single-workgroup finalize
// kernels (one thread), read by the streaming kernels at their start.
struct alignas(64) Scalars {
    double rho, rho_prev, alpha, omega, beta;
    double rr;          // ||r||^2
    double rhat2;       // ||rhat||^2
    double nb2;         // ||b||^2 of the system this run solves
    double thr2;        // tol^2 * ||b||^2
    double ss;          // ||s||^2 of the current iteration
    double last_rel;    // last recursive relative residual
    double eps_bd;      // breakdown threshold (relative cosine)
    double aux0;        // tolerance of this run (read by FIN_INIT)
    double net_q2;      // learned preconditioner: ||q||^2 of its input
    double net_z2;      //   ||T^{-1} q||^2
    double net_ee;      //   ||e||^2 of the training target
    int iter;           // iterations completed in this run
    int maxit;
    int done;           // 1: nothing more to do (status says why)
    int status;         // 0 converged, 1 iteration limit, 2 breakdown, 4 periodic restart due
    int fresh;          // 1: the next iteration restarts (rhat = r, p = r)
    int was_fresh;      // the current iteration started fresh
    int skip;           // sigma breakdown: rest of the current iteration is skipped
    int half;           // converged at the half step of the current iteration
    int wbd;            // omega breakdown in the current iteration
    int restarts;
    int restart_every;
    int hist_base;      // first history slot of this run
    int hist_cap;
    int work_mask;      // streaming kernels of the last iteration that did work (bit = eg_kernel)
    int pad[2];
};

// Views of one precision set of the operator.
template <typename Tc> struct CoefTraits;
template <> struct CoefTraits<double> { using val = double; static constexpr bool quant = false; };
template <> struct CoefTraits<float> { using val = float; static constexpr bool quant = false; };
struct bf16_t { uint16_t bits; };
struct fp16_t { uint16_t bits; };
template <> struct CoefTraits<bf16_t> { using val = float; static constexpr bool quant = true; };
template <> struct CoefTraits<fp16_t> { using val = float; static constexpr bool quant = true; };

// floats per (level, latitude row) record of a 16-bit coefficient set: the six directions'
// power-of-two scales at 0..5 and their offsets at 8..13 (a coupling is offset + q * scale)
constexpr int kQsStride = 16;
constexpr int kQsOff = 8;

template <typename Tc> struct OpView {
    using V = typename CoefTraits<Tc>::val;
    const Tc *a;        // [6][n]
    const V *m;         // [n]
    const float *qs;    // [nlev][nlat][kQsStride] scales and offsets (16-bit sets only)
    int nlon, nlat, nlev;
    long P, n;
};

// Factors of the vertical tridiagonal: f[3][n] = (l, inv, c), see k_tri_factor.
template <typename Tv> struct TriView {
    const Tv *f;
    long P, n;
    int nlev;
};

// flags a streaming kernel may be told to stop on
constexpr int STOP_DONE = 1, STOP_SKIP = 2, STOP_HALF = 4;

// ---- launchers (kernels.hip) ----
// rows of the partial-sum buffer the kernels of a grid of this shape may write
int partial_rows_needed(int nlon, int nlat, int nlev);
// SpMV variants.  w is the dot partner; partials receive one row per workgroup.
enum SpmvMode { SP_PLAIN = 0, SP_DOT2 = 1 };
template <typename Tv, typename Tc>
void launch_spmv(const OpView<Tc> &op, const Tv *x, Tv *y, const Tv *w, int mode, double *partials,
                 int *nrows, const Scalars *sc, int stop_mask, hipStream_t s);
// r = b - A x in FP64 with the result written as Tout; partials: ||r64||^2, ||b||^2, ||rout||^2
template <typename Tout>
void launch_residual(const OpView<double> &op, const double *b, const double *x, Tout *r, double *partials,
                     int *nrows, hipStream_t s);

// TH_PF: the TH_P step of an iteration that starts afresh (rhat = p = r), a kernel of its own on
// the register path (launched beside TH_P; each returns at once unless the device's restart
// flag says it is the one)
enum ThomasMode { TH_PLAIN = 0, TH_P = 1, TH_S = 2, TH_PF = 3 };
// stop_mask: flags that make a TH_PLAIN launch return at once (TH_P / TH_S use their own)
template <typename Tv>
void launch_thomas(const TriView<Tv> &tv, const Tv *q, Tv *z, int mode, const Tv *r, Tv *p, const Tv *v, Tv *rhat,
                   double *partials, int *nrows, const Scalars *sc, hipStream_t s, int stop_mask = 0);
// The same with the result zcm = T^{-1} q, and q itself (qcm), written in the colour-major
// order of the line-SOR kernels (nlon even): the start of a line-SOR application.
template <typename Tv>
void launch_thomas_cm(const TriView<Tv> &tv, int nlon, const Tv *q, Tv *zcm, Tv *qcm, int mode, const Tv *r, Tv *p,
                      const Tv *v, Tv *rhat, double *partials, int *nrows, const Scalars *sc, hipStream_t s,
                      int stop_mask = 0);
// Red-black vertical-line SOR.  SorView: the LU factors of T (f[3]) and the W, E, S, N
// couplings (a[4]) in colour-major order (index colour * n/2 + k * P/2 + j * nlon/2 + i/2).
template <typename Tv, typename Tc> struct SorView {
    const Tv *f;
    const Tc *a;
};
// reorder nd arrays of n values from grid order into colour-major order (nlon even)
template <typename T> void launch_sor_perm(const T *src, T *dst, int nd, int nlon, int nlat, int nlev, hipStream_t s);
// `sweeps` sweeps with relaxation omega applied to q.  qcm: q in colour-major order; xcm: T^{-1} q
// in colour-major order on entry (launch_thomas_cm writes both), overwritten; wsc: n/2 values of
// scratch; xout: the result in grid order.
template <typename Tv, typename Tc>
void launch_sor(const OpView<Tc> &op, const SorView<Tv, Tc> &sv, const Tv *qcm, Tv *xcm, Tv *wsc, Tv *xout,
                int sweeps, double omega, const Scalars *sc, int stop_mask, hipStream_t s);
template <typename Tf>
void launch_tri_factor(const double *a64, const double *m64, int nlon, int nlat, int nlev, Tf *f, hipStream_t s);

// x (FP64) += alpha phat + omega shat; r = s - omega t (FP32): the paper's mixed-precision update
// (x32: x rounded to FP32 after every update, the all-32-bit solver)
void launch_update_mp(long n, double *x, const float *ph, const float *sh, const float *s, const float *t, float *r,
                      const float *rhat, double *partials, int *nrows, const Scalars *sc, bool x32, hipStream_t stream);
template <typename Tv>
void launch_update(long n, Tv *x, const Tv *ph, const Tv *sh, const Tv *s, const Tv *t, Tv *r, const Tv *rhat,
                   double *partials, int *nrows, const Scalars *sc, hipStream_t stream);

template <typename Ta, typename Tb>
void launch_dot(long n, const Ta *a, const Tb *b, double *partials, int *nrows, hipStream_t s);
// partial columns 0 and 1: <a, b> and <c, d> (FP64 products and sums)
template <typename T>
void launch_dot2(long n, const T *a, const T *b, const T *c, const T *d, double *partials, int *nrows,
                 const Scalars *sc, int stop_mask, hipStream_t s);

// FGMRES: blocked classical Gram-Schmidt over basis vectors V + i * n (kMBlk per pass).
// launch_mdot writes <w, v_{i0+c}> to out[i0 + c]; part must hold elementwise rows x kMBlk.
constexpr int kMBlk = 8;
template <typename Tv>
int launch_mdot(long n, const Tv *w, const Tv *V, int i0, int nb, double *part, double *out, hipStream_t s);
template <typename Tv>
int launch_maxpy(long n, Tv *w, const Tv *V, int i0, int nb, const double *h, double sign, int want_norm,
                 double *part, hipStream_t s);
template <typename Tv> void launch_vscale(long n, const Tv *x, Tv *y, const double *d, hipStream_t s);

// finalize kernels (one workgroup): reduce partials, update the scalar block
enum FinStage { FIN_INIT = 0, FIN_END = 1, FIN_SIGMA = 2, FIN_S = 3, FIN_OMEGA = 4, FIN_SUM = 5, FIN_TRUE = 6,
                FIN_NET = 7, FIN_LOSS = 8 };
// c_rr / c_nb: partial columns holding ||r||^2 and ||b||^2 (FIN_INIT, FIN_TRUE)
void launch_finalize(int stage, const double *partials, int nrows, Scalars *sc, double *hist, double *out,
                     int c_rr, int c_nb, hipStream_t s);

template <typename T> void launch_fill(T *p, long n, T v, hipStream_t s);
void launch_add_correction(long n, double *x, const float *d, hipStream_t s);
void launch_sub_to_f32(long n, const double *a, const double *b, float *out, hipStream_t s);
void launch_cast_f32(long n, const double *a, float *out, hipStream_t s);

// operator setup
void launch_derive(const double *coeffs, int nlon, int nlat, int nlev, double *a64, double *m64, int *bad,
                   hipStream_t s);
void launch_to_fp32(long n, const double *a64, const double *m64, float *a32, float *m32, hipStream_t s);
void launch_quantize(int kind, int nlon, int nlat, int nlev, const double *a64, uint16_t *aq, float *qs,
                     hipStream_t s);
void launch_check_finite(long n, const double *v, int *bad, hipStream_t s);

// ---- learned preconditioner (net.hip) ----
// flat parameter vector: W1[5][32][4] b1[32] W2[9][32][32] b2[32] W3[5][32][32] b3[32] W4[5][32] b4
constexpr int kNetParams = 15233;
constexpr int kNetOffW1 = 0, kNetOffB1 = 640, kNetOffW2 = 672, kNetOffB2 = 9888, kNetOffW3 = 9920,
              kNetOffB3 = 15040, kNetOffW4 = 15072, kNetOffB4 = 15232;
constexpr int kNetPartRows = 768;   // rows of per-workgroup partial weight gradients (3 per CU)

struct NetGeo {
    int nlon, nlat, nlev;
    long P, n;
};

// device state of one network: FP32 master weights, gradient, Adam moments, and the BF16
// copies the MFMA kernels read (w1f [co][tap*4+ci] padded to 32, w2f/w3f [tap][co][ci],
// w2b/w3b [tap][ci][co] for the transposed convolutions, w4 as BF16-rounded floats)
struct NetDev {
    float *theta, *grad, *adam_m, *adam_v, *part;
    uint16_t *w1f, *w2f, *w3f, *w2b, *w3b;
    float *w4;
};

// activations of one application: x0 [n][4], a1..a3 [n][32] (BF16); d1, d2 [n][32] BF16
// gradient buffers (training only)
struct NetActs {
    uint16_t *x0, *a1, *a2, *a3, *d1, *d2;
};

template <typename Tv, typename Tc>
void launch_net_features(const NetGeo &g, const Tv *q, const Tv *z0, const Tc *a, uint16_t *x0, const Scalars *sc,
                         int stop_mask, hipStream_t s);
void launch_net_forward_layers(const NetGeo &g, const NetDev &d, const NetActs &act, const Scalars *sc, int stop_mask,
                               hipStream_t s);
// inference: layers 1-2, then layer 3 fused with the output layer (a3 is not stored)
template <typename Tv>
void launch_net_forward_fused(const NetGeo &g, const NetDev &d, const NetActs &act, const Tv *q, Tv *qout,
                              float *delta, const Scalars *sc, int stop_mask, hipStream_t s);
// inference in one launch (grids with nlon a multiple of 64, net_fused_ok): input channels
// from q, z0 = T^{-1} q and the operator's static channels (launch_net_static, one BF16 pair
// per point), every layer, and q' = q + rho delta; bitwise the layered path's result
bool net_fused_ok(const NetGeo &g);
void launch_net_static(long n, const double *a64, uint32_t *fs, hipStream_t s);
template <typename Tv>
void launch_net_infer(const NetGeo &g, const NetDev &d, const Tv *q, const Tv *z0, const uint32_t *fstat, Tv *qout,
                      float *delta, const Scalars *sc, int stop_mask, hipStream_t s);
template <typename Tv>
void launch_net_out(const NetGeo &g, const NetDev &d, const NetActs &act, const Tv *q, Tv *qout, float *delta,
                    const Scalars *sc, int stop_mask, hipStream_t s);
void launch_thomas_t(const TriView<float> &tv, const float *y, float *z, hipStream_t s);
void launch_spmv_t(const NetGeo &g, const float *a, const float *m, const float *x, float *y, hipStream_t s);
void launch_net_gseed(long n, const float *m, const float *e, float *g, const Scalars *sc, hipStream_t s);
void launch_net_diff(long n, const float *m, const float *e, float *out, hipStream_t s);
void launch_net_backward(const NetGeo &g, const NetDev &d, const NetActs &act, const float *u, const Scalars *sc,
                         int first, hipStream_t s);
void launch_net_grad(const NetDev &d, float scale, hipStream_t s);
void launch_net_refresh(const NetDev &d, hipStream_t s);
void launch_net_adam(const NetDev &d, float lr, int step, hipStream_t s);

}  // namespace eg
