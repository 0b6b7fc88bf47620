// Host side of the endgame library: operator object, BiCGStab drivers and the C ABI.
//
// BiCGStab (Sec. 2, Eq. 5 of the paper: right-preconditioned, so the tracked residual is the
// unpreconditioned b - A x that the halting test of Sec. 3, Eq. 8-9 measures) runs as a
// device-driven state machine: the streaming kernels read alpha, beta, omega and the flags
// from a device scalar block, single-workgroup finalize kernels reduce the FP64 partials and
// advance the recurrences.  The host only enqueues batches of iterations and looks at the
// flags between batches; kernels enqueued after convergence return at once, so the stopping
// iteration is exact.
//
// One iteration (kernel order):
//   thomas(P)  p = r + beta (p - omega v); phat = T^{-1} p
//   spmv       v = A phat;  <rhat, v>, <v, v>               -> finalize(SIGMA): alpha
//   thomas(S)  s = r - alpha v; shat = T^{-1} s; <s, s>    -> finalize(S): half-step exit?
//   spmv       t = A shat;  <t, s>, <t, t>                  -> finalize(OMEGA): omega
//   update     x += alpha phat + omega shat; r = s - omega t; <rhat, r>, <r, r>
//                                                           -> finalize(END): rho, beta, stop?
//
// Mixed precision (Sec. 3-4 of the paper keep x in 64-bit, do the bulk in 32-bit and revert
// the global sums to 64-bit): the refinement driver forms r = b - A x in FP64, rounds it to
// FP32, solves A d = r with the FP32 machine above (FP64 dot accumulation) to a modest
// relative tolerance eta, and updates x += d in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/endgame.h"
#include "eg_internal.h"

using namespace eg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define EG_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(EG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T> int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(EG_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    return 0;
}

template <typename T> void dfree(T *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

constexpr int kMaxGmres = 64;   // largest FGMRES restart length

template <typename Tv> struct Fgm {   // FGMRES basis storage of one precision
    Tv *V = nullptr, *Z = nullptr, *W = nullptr, *R = nullptr, *tmp = nullptr;
    int m = 0;
};

template <typename Tv> struct Work {
    Tv *r = nullptr, *rh = nullptr, *p = nullptr, *ph = nullptr, *v = nullptr, *s = nullptr, *sh = nullptr,
       *t = nullptr, *x = nullptr;
    Tv *qp = nullptr;   // learned modes: q + rho * delta before the final tridiagonal solve
    bool ready = false;
};

// ---- allocation-free inner product (eg_dot_noalloc) ----------------------------------------
// Its per-workgroup partial sums (at most kNoAllocRows rows, the row count of the elementwise
// kernels) and its result live in this file-scope device array: one copy per GPU, held until
// the process ends.  Host code must not pass the array's name to a kernel (on the host it is a
// stand-in, not a device address): it uses the address hipGetSymbolAddress returns for the
// current device, looked up once per device.
constexpr int kNoAllocRows = 8192;
constexpr int kNoAllocDoubles = kNoAllocRows * kPartialCols + kPartialCols;
constexpr long kNoAllocMaxN = 1L << 40;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
int scratch_ptr(double **out)
{
    int dev = 0;
    EG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(EG_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        EG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

}  // namespace

// The learned preconditioner's network: weights, optimiser state, activation and training
// buffers (grown to the largest grid used).
struct eg_net {
    NetDev d{};
    NetActs act{};
    long act_cap = 0;
    bool act_train = false;
    float *t_z0 = nullptr, *t_qp = nullptr, *t_m = nullptr, *t_diff = nullptr, *t_g = nullptr, *t_u = nullptr;
    long t_cap = 0;
    double *d_loss = nullptr;   // per-pair losses of the current pass
    long loss_cap = 0;
    int step = 0;               // Adam steps taken
    int loss_kind = 1;          // 0: ||M(r) - e||^2 / ||e||^2,  1: ||A M(r) - r||^2 / ||r||^2
};

// A batch of plain iterations captured as a HIP graph, with everything its kernels were
// launched with: the same key means the same launches, so the graph can be replayed.
struct IterKey {
    const void *a, *m, *qs, *tri, *sor_ws, *sorf, *sora, *mp_x, *partials, *sc, *hist;
    const void *w[9];
    int tv, tc, sor_on, sweeps, mp_active, mp_x32, batch;
    double omega;
};
struct IterGraph {
    IterKey key;
    hipGraphExec_t exec;
};

struct eg_operator {
    int nlon = 0, nlat = 0, nlev = 0;
    long P = 0, n = 0;
    hipStream_t stream = nullptr;

    double *a64 = nullptr, *m64 = nullptr, *tri64 = nullptr;
    float *a32 = nullptr, *m32 = nullptr, *tri32 = nullptr;
    uint16_t *aq[2] = {nullptr, nullptr};
    float *qs[2] = {nullptr, nullptr};

    Work<double> w64;
    Work<float> w32;

    double *partials = nullptr;
    Scalars *sc = nullptr;       // device
    Scalars *h_sc = nullptr;     // pinned host mirror
    double *d_out = nullptr;     // device, 4 doubles
    double *h_out = nullptr;     // pinned host, 4 doubles
    int *d_bad = nullptr;        // device, 4 ints
    double *d_hist = nullptr;
    int hist_cap = 0;

    double eta = 1e-2;          // inner relative tolerance of one refinement step
    int restart_every = 0;
    int max_outer = 30;
    int inner_maxit = 1000;     // iterations of one inner FP32 solve of the refinement
    int poll = 8;
    int stall_window = 20;
    double eps_bd = 2.220446049250313e-16;   // breakdown threshold (relative cosine), 2^-52
    int precond = 0;            // plain modes: 0 T^{-1}, 1 red-black vertical-line SOR
    int sor_sweeps = 3;
    double sor_omega = 1.5;
    bool sor_on = false;        // SOR active in the current solve (plain modes with precond 1)
    // line-SOR work vectors in colour-major order: x (n), q (n) and the parked forward
    // values (n/2), room for FP64 (5n/2 doubles)
    double *sor_ws = nullptr;
    double *mp_x = nullptr;     // EG_FP32_MP: the FP64 solution the FP32 iteration updates
    double *ir_backup = nullptr;   // refinement: x before the last correction
    bool mp_active = false;
    bool mp_x32 = false;        // EG_FP32_MP with the solution held in 32 bits too (option mp_x32)
    // colour-major copies of the LU factors and the W, E, S, N couplings the SOR reads
    double *sorf64 = nullptr, *sora64 = nullptr;
    float *sorf32 = nullptr, *sora32 = nullptr;
    uint16_t *sorq[2] = {nullptr, nullptr};
    int profile = 0;
    int use_graph = 1;          // replay the batched iteration as a HIP graph (option graph)
    hipStream_t cap_stream = nullptr;   // private stream the graphs are captured on
    std::vector<IterGraph> graphs;      // instantiated iteration batches, newest last

    // kernel timing: events around the streaming kernels of one iteration + the residual
    hipEvent_t ev[16] = {};
    bool ev_ready = false;
    double kms[EG_K_COUNT][4] = {};
    long kcnt[EG_K_COUNT][4] = {};

    eg_info info{};
    std::vector<double> hist_host;
    int hist_count = 0;
    eg_net *net = nullptr;      // learned preconditioner of the learned modes (own_net or a caller's)
    eg_net *own_net = nullptr;  // network owned by the operator (eg_train/load_learned_pc)
    uint32_t *net_fs = nullptr; // static input channels of the one-launch inference (BF16 pairs)
    int net_fused = 1;          // 0: the layered inference (kept for comparison)
    double *harvest_x = nullptr;
    int method = 0;             // plain modes: 0 BiCGStab, 1 FGMRES
    int learned_method = 1;     // learned modes: 0 flexible BiCGStab, 1 FGMRES
    int gm_m = 30;              // FGMRES restart length
    Fgm<double> f64;
    Fgm<float> f32;
    double *d_h = nullptr;      // FGMRES: Gram-Schmidt coefficients (two passes) / solution weights
    double *mpart = nullptr;    // FGMRES: partial sums of the blocked dot products
    double *h_h = nullptr;      // pinned host mirror of d_h
    std::vector<double> hist_pending;   // history written on the host (FGMRES)
    template <typename Tv> Fgm<Tv> &fgm()
    {
        if constexpr (std::is_same_v<Tv, double>) return f64;
        else return f32;
    }

    OpView<double> view64() const { return {a64, m64, nullptr, nlon, nlat, nlev, P, n}; }
    OpView<float> view32() const { return {a32, m32, nullptr, nlon, nlat, nlev, P, n}; }
    template <typename Tq> OpView<Tq> viewq(int slot) const
    {
        return {reinterpret_cast<const Tq *>(aq[slot]), m32, qs[slot], nlon, nlat, nlev, P, n};
    }
    template <typename Tv> Tv *sor_x() const { return reinterpret_cast<Tv *>(sor_ws); }
    template <typename Tv> Tv *sor_q() const { return reinterpret_cast<Tv *>(sor_ws) + n; }
    template <typename Tv> Tv *sor_w() const { return reinterpret_cast<Tv *>(sor_ws) + 2 * n; }
    template <typename Tv, typename Tc> SorView<Tv, Tc> sor_view() const
    {
        if constexpr (std::is_same_v<Tc, double>) return {sorf64, sora64};
        else if constexpr (std::is_same_v<Tc, float>) return {sorf32, sora32};
        else if constexpr (std::is_same_v<Tc, bf16_t>) return {sorf32, reinterpret_cast<const bf16_t *>(sorq[0])};
        else return {sorf32, reinterpret_cast<const fp16_t *>(sorq[1])};
    }
    TriView<double> tri_view64() const { return {tri64, P, n, nlev}; }
    TriView<float> tri_view32() const { return {tri32, P, n, nlev}; }
    // the Thomas factors a precision uses: FP64, or FP32 for every lower-precision set
    template <typename Tv> TriView<Tv> tri_view() const
    {
        if constexpr (std::is_same_v<Tv, double>) return tri_view64();
        else return tri_view32();
    }
};

namespace {

int ensure_fp32(eg_operator *op)
{
    if (op->a32) return 0;
    int rc;
    if ((rc = dalloc(&op->a32, 6 * (size_t)op->n))) return rc;
    if ((rc = dalloc(&op->m32, (size_t)op->n))) return rc;
    if ((rc = dalloc(&op->tri32, 3 * (size_t)op->n))) return rc;
    launch_to_fp32(op->n, op->a64, op->m64, op->a32, op->m32, op->stream);
    launch_tri_factor<float>(op->a64, op->m64, op->nlon, op->nlat, op->nlev, op->tri32, op->stream);
    EG_HIP(hipGetLastError());
    return 0;
}

int ensure_quant(eg_operator *op, int kind)
{
    const int slot = (kind == PBF16) ? 0 : 1;
    int rc;
    if ((rc = ensure_fp32(op))) return rc;   // m32 and the FP32 factors are shared with the FP32 set
    if (op->aq[slot]) return 0;
    if ((rc = dalloc(&op->aq[slot], 6 * (size_t)op->n))) return rc;
    if ((rc = dalloc(&op->qs[slot], (size_t)kQsStride * op->nlev * op->nlat))) return rc;
    launch_quantize(kind, op->nlon, op->nlat, op->nlev, op->a64, op->aq[slot], op->qs[slot], op->stream);
    EG_HIP(hipGetLastError());
    return 0;
}

// the colour-major constants of the red-black line SOR for one coefficient set
template <typename Tc> int ensure_sor(eg_operator *op)
{
    int rc;
    const size_t n = (size_t)op->n;
    hipStream_t s = op->stream;
    if (!op->sor_ws && (rc = dalloc(&op->sor_ws, n * 5 / 2))) return rc;
    if constexpr (std::is_same_v<Tc, double>) {
        if (op->sorf64) return 0;
        if ((rc = dalloc(&op->sorf64, 3 * n)) || (rc = dalloc(&op->sora64, 4 * n))) return rc;
        launch_sor_perm<double>(op->tri64, op->sorf64, 3, op->nlon, op->nlat, op->nlev, s);
        launch_sor_perm<double>(op->a64, op->sora64, 4, op->nlon, op->nlat, op->nlev, s);
    } else {
        if ((rc = ensure_fp32(op))) return rc;
        if (!op->sorf32) {
            if ((rc = dalloc(&op->sorf32, 3 * n))) return rc;
            launch_sor_perm<float>(op->tri32, op->sorf32, 3, op->nlon, op->nlat, op->nlev, s);
        }
        if constexpr (std::is_same_v<Tc, float>) {
            if (op->sora32) return 0;
            if ((rc = dalloc(&op->sora32, 4 * n))) return rc;
            launch_sor_perm<float>(op->a32, op->sora32, 4, op->nlon, op->nlat, op->nlev, s);
        } else {
            const int slot = std::is_same_v<Tc, bf16_t> ? 0 : 1;
            if ((rc = ensure_quant(op, slot == 0 ? PBF16 : PFP16))) return rc;
            if (op->sorq[slot]) return 0;
            if ((rc = dalloc(&op->sorq[slot], 4 * n))) return rc;
            launch_sor_perm<uint16_t>(op->aq[slot], op->sorq[slot], 4, op->nlon, op->nlat, op->nlev, s);
        }
    }
    EG_HIP(hipGetLastError());
    return 0;
}

template <typename Tv> int ensure_work(eg_operator *op, Work<Tv> &w)
{
    if (w.ready) return 0;
    Tv **bufs[] = {&w.r, &w.rh, &w.p, &w.ph, &w.v, &w.s, &w.sh, &w.t, &w.x};
    for (Tv **b : bufs) {
        int rc = dalloc(b, (size_t)op->n);
        if (rc) return rc;
    }
    w.ready = true;
    return 0;
}

int ensure_hist(eg_operator *op, int cap)
{
    if (cap <= op->hist_cap) return 0;
    dfree(op->d_hist);
    int rc = dalloc(&op->d_hist, (size_t)cap);
    if (rc) return rc;
    op->hist_cap = cap;
    return 0;
}

int sync_scalars(eg_operator *op)
{
    EG_HIP(hipMemcpyAsync(op->h_sc, op->sc, sizeof(Scalars), hipMemcpyDeviceToHost, op->stream));
    EG_HIP(hipStreamSynchronize(op->stream));
    return 0;
}

// Set the run parameters of the scalar block (host fields) before FIN_INIT.
int put_run_params(eg_operator *op, double tol, int maxit, int hist_base, int restart_every)
{
    Scalars h{};
    h.aux0 = tol;
    h.maxit = maxit;
    h.eps_bd = op->eps_bd;
    h.hist_base = hist_base;
    h.hist_cap = op->hist_cap;
    h.restart_every = restart_every;
    *op->h_sc = h;
    EG_HIP(hipMemcpyAsync(op->sc, op->h_sc, sizeof(Scalars), hipMemcpyHostToDevice, op->stream));
    return 0;
}

template <typename Tc> constexpr int prec_of()
{
    if constexpr (std::is_same_v<Tc, double>) return EG_PREC_FP64;
    else if constexpr (std::is_same_v<Tc, float>) return EG_PREC_FP32;
    else if constexpr (std::is_same_v<Tc, bf16_t>) return EG_PREC_BF16;
    else return EG_PREC_FP16;
}

int ensure_events(eg_operator *op)
{
    if (op->ev_ready) return 0;
    for (hipEvent_t &e : op->ev) EG_HIP(hipEventCreate(&e));
    op->ev_ready = true;
    return 0;
}

// Accumulate the device time between event pair k (events 2k, 2k+1) into kernel `kind`.
int add_kernel_time(eg_operator *op, int k, int kind, int prec)
{
    float ms = 0.f;
    EG_HIP(hipEventElapsedTime(&ms, op->ev[2 * k], op->ev[2 * k + 1]));
    op->kms[kind][prec] += ms;
    op->kcnt[kind][prec] += 1;
    return 0;
}

// ev (may be null): 10 events recorded around the five streaming kernels.
template <typename Tv, typename Tc>
void enqueue_iteration(eg_operator *op, const OpView<Tc> &A, Work<Tv> &w, hipEvent_t *ev)
{
    hipStream_t s = op->stream;
    const TriView<Tv> T = op->tri_view<Tv>();
    int nr = 0;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    const bool sor = op->sor_on;
    Tv *xcm = sor ? op->sor_x<Tv>() : nullptr, *qcm = sor ? op->sor_q<Tv>() : nullptr;
    Tv *wsc = sor ? op->sor_w<Tv>() : nullptr;
    mark(0);
    if (sor)
        launch_thomas_cm<Tv>(T, op->nlon, nullptr, xcm, qcm, TH_P, w.r, w.p, w.v, w.rh, op->partials, &nr, op->sc, s);
    else
        launch_thomas<Tv>(T, nullptr, w.ph, TH_P, w.r, w.p, w.v, w.rh, op->partials, &nr, op->sc, s);
    mark(1);
    if (sor) {
        mark(12);
        launch_sor<Tv, Tc>(A, op->sor_view<Tv, Tc>(), qcm, xcm, wsc, w.ph, op->sor_sweeps, op->sor_omega, op->sc,
                           STOP_DONE, s);
        mark(13);
    }
    mark(2);
    launch_spmv<Tv, Tc>(A, w.ph, w.v, w.rh, SP_DOT2, op->partials, &nr, op->sc, STOP_DONE, s);
    mark(3);
    launch_finalize(FIN_SIGMA, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
    mark(4);
    if (sor)
        launch_thomas_cm<Tv>(T, op->nlon, nullptr, xcm, qcm, TH_S, w.r, w.s, w.v, nullptr, op->partials, &nr, op->sc, s);
    else
        launch_thomas<Tv>(T, nullptr, w.sh, TH_S, w.r, w.s, w.v, nullptr, op->partials, &nr, op->sc, s);
    mark(5);
    launch_finalize(FIN_S, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
    if (sor) {
        mark(14);
        launch_sor<Tv, Tc>(A, op->sor_view<Tv, Tc>(), qcm, xcm, wsc, w.sh, op->sor_sweeps, op->sor_omega, op->sc,
                           STOP_DONE | STOP_SKIP | STOP_HALF, s);
        mark(15);
    }
    mark(6);
    launch_spmv<Tv, Tc>(A, w.sh, w.t, w.s, SP_DOT2, op->partials, &nr, op->sc, STOP_DONE | STOP_SKIP | STOP_HALF, s);
    mark(7);
    launch_finalize(FIN_OMEGA, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
    mark(8);
    if constexpr (std::is_same_v<Tv, float>) {
        if (op->mp_active)
            launch_update_mp(op->n, op->mp_x, w.ph, w.sh, w.s, w.t, w.r, w.rh, op->partials, &nr, op->sc, op->mp_x32,
                             s);
        else
            launch_update<Tv>(op->n, w.x, w.ph, w.sh, w.s, w.t, w.r, w.rh, op->partials, &nr, op->sc, s);
    } else {
        launch_update<Tv>(op->n, w.x, w.ph, w.sh, w.s, w.t, w.r, w.rh, op->partials, &nr, op->sc, s);
    }
    mark(9);
    launch_finalize(FIN_END, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
}

// `batch` plain iterations as one HIP graph: found among the operator's graphs by what its
// launches read, else captured on the private stream and instantiated.  The iteration is
// kernel launches only (no memset or copy nodes), and every kernel takes its per-iteration
// decisions from the device scalar block, so a replay does what eager launches would.
template <typename Tv, typename Tc>
int iteration_graph(eg_operator *op, const OpView<Tc> &A, Work<Tv> &w, int batch, hipGraphExec_t *out)
{
    IterKey key;
    std::memset(&key, 0, sizeof key);
    key.a = A.a;
    key.m = A.m;
    key.qs = A.qs;
    key.tri = op->tri_view<Tv>().f;
    key.sor_on = op->sor_on;
    if (op->sor_on) {
        const SorView<Tv, Tc> sv = op->sor_view<Tv, Tc>();
        key.sor_ws = op->sor_ws;
        key.sorf = sv.f;
        key.sora = sv.a;
        key.sweeps = op->sor_sweeps;
        key.omega = op->sor_omega;
    }
    key.mp_active = op->mp_active;
    key.mp_x32 = op->mp_x32;
    key.mp_x = op->mp_active ? op->mp_x : nullptr;
    key.partials = op->partials;
    key.sc = op->sc;
    key.hist = op->d_hist;
    const void *wv[9] = {w.r, w.rh, w.p, w.ph, w.v, w.s, w.sh, w.t, w.x};
    for (int i = 0; i < 9; ++i) key.w[i] = wv[i];
    key.tv = sizeof(Tv);
    key.tc = prec_of<Tc>();
    key.batch = batch;
    for (const IterGraph &g : op->graphs)
        if (std::memcmp(&g.key, &key, sizeof key) == 0) {
            *out = g.exec;
            return 0;
        }
    if (!op->cap_stream) EG_HIP(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking));
    EG_HIP(hipGetLastError());
    EG_HIP(hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipStream_t user = op->stream;
    op->stream = op->cap_stream;
    for (int b = 0; b < batch; ++b) enqueue_iteration<Tv, Tc>(op, A, w, nullptr);
    op->stream = user;
    hipGraph_t graph = nullptr;
    const hipError_t launched = hipGetLastError();
    const hipError_t ended = hipStreamEndCapture(op->cap_stream, &graph);
    if (launched != hipSuccess || ended != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(EG_EHIP, std::string("capture of the iteration failed: ") +
                                 hipGetErrorString(launched != hipSuccess ? launched : ended));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (inst != hipSuccess) return fail(EG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(inst));
    if (op->graphs.size() >= 8) {   // a few modes per operator; drop the oldest
        (void)hipGraphExecDestroy(op->graphs.front().exec);
        op->graphs.erase(op->graphs.begin());
    }
    op->graphs.push_back({key, exec});
    *out = exec;
    return 0;
}

// Run Krylov iterations until the device says done.  Precondition: FIN_INIT (or FIN_TRUE) has
// been enqueued for this run; w.r holds the residual and w.x the iterate.
template <typename Tv, typename Tc> int krylov_run(eg_operator *op, const OpView<Tc> &A, Work<Tv> &w)
{
    int rc;
    if ((rc = sync_scalars(op))) return rc;
    if (op->profile) {
        // one iteration per check; time the streaming kernels that did work
        if ((rc = ensure_events(op))) return rc;
        constexpr int prec = prec_of<Tc>();
        while (!op->h_sc->done) {
            enqueue_iteration<Tv, Tc>(op, A, w, op->ev);
            EG_HIP(hipGetLastError());
            if ((rc = sync_scalars(op))) return rc;
            const int mask = op->h_sc->work_mask;
            for (int k = 0; k < 5; ++k)
                if (mask & (1 << k))
                    if ((rc = add_kernel_time(op, k, k, prec))) return rc;
            if (op->sor_on) {
                if ((mask & 1) && (rc = add_kernel_time(op, 6, EG_K_SOR_P, prec))) return rc;
                if ((mask & 4) && (rc = add_kernel_time(op, 7, EG_K_SOR_S, prec))) return rc;
            }
        }
        return 0;
    }
    int batch = std::max(1, op->poll);
    if (op->use_graph) {
        hipGraphExec_t exec = nullptr;
        if ((rc = iteration_graph<Tv, Tc>(op, A, w, batch, &exec))) return rc;
        while (!op->h_sc->done) {
            EG_HIP(hipGraphLaunch(exec, op->stream));
            if ((rc = sync_scalars(op))) return rc;
        }
        return 0;
    }
    while (!op->h_sc->done) {
        for (int b = 0; b < batch; ++b) enqueue_iteration<Tv, Tc>(op, A, w, nullptr);
        EG_HIP(hipGetLastError());
        if ((rc = sync_scalars(op))) return rc;
    }
    return 0;
}

// ---- learned preconditioner ---------------------------------------------------------------
int ensure_acts(eg_net *net, long n, bool train)
{
    if (n <= net->act_cap && (!train || net->act_train)) return 0;
    const long cap = std::max(n, net->act_cap);
    NetActs &a = net->act;
    dfree(a.x0); dfree(a.a1); dfree(a.a2); dfree(a.a3); dfree(a.d1); dfree(a.d2);
    net->act_cap = 0;
    int rc;
    if ((rc = dalloc(&a.x0, 4 * (size_t)cap)) || (rc = dalloc(&a.a1, 32 * (size_t)cap)) ||
        (rc = dalloc(&a.a2, 32 * (size_t)cap)) || (rc = dalloc(&a.a3, 32 * (size_t)cap)))
        return rc;
    if (train || net->act_train) {
        if ((rc = dalloc(&a.d1, 32 * (size_t)cap)) || (rc = dalloc(&a.d2, 32 * (size_t)cap))) return rc;
        net->act_train = true;
    }
    net->act_cap = cap;
    return 0;
}

int ensure_train_tmp(eg_net *net, long n)
{
    if (n <= net->t_cap) return 0;
    float **bufs[] = {&net->t_z0, &net->t_qp, &net->t_m, &net->t_diff, &net->t_g, &net->t_u};
    for (float **b : bufs) {
        dfree(*b);
        int rc = dalloc(b, (size_t)n);
        if (rc) return rc;
    }
    net->t_cap = n;
    return 0;
}

template <typename Tv> int ensure_qp(eg_operator *op, Work<Tv> &w)
{
    return w.qp ? 0 : dalloc(&w.qp, (size_t)op->n);
}

NetGeo geo_of(const eg_operator *op);

// the static input channels of the one-launch inference, built once per operator from the
// FP64 couplings (their FP32 roundings give the same channels)
int ensure_net_static(eg_operator *op)
{
    if (op->net_fs || !net_fused_ok(geo_of(op))) return 0;
    int rc = dalloc(&op->net_fs, (size_t)op->n);
    if (rc) return rc;
    launch_net_static(op->n, op->a64, op->net_fs, op->stream);
    EG_HIP(hipGetLastError());
    return 0;
}

NetGeo geo_of(const eg_operator *op) { return {op->nlon, op->nlat, op->nlev, op->P, op->n}; }

// z (holding T^{-1} q on entry) <- M(q) = T^{-1} (q + rho delta(q)).  Tc: coefficient set the
// input channels are read from.
template <typename Tv, typename Tc>
void enqueue_net_stage(eg_operator *op, eg_net *net, const Tc *coef, const Tv *q, Tv *z, Tv *qp, float *delta,
                       int stop_mask)
{
    hipStream_t s = op->stream;
    const NetGeo g = geo_of(op);
    int nr = 0;
    launch_dot2<Tv>(op->n, q, q, z, z, op->partials, &nr, op->sc, stop_mask, s);
    launch_finalize(FIN_NET, op->partials, nr, op->sc, nullptr, nullptr, 0, 0, s);
    if (op->net_fs && op->net_fused) {
        launch_net_infer<Tv>(g, net->d, q, z, op->net_fs, qp, delta, op->sc, stop_mask, s);
    } else {
        launch_net_features<Tv, Tc>(g, q, z, coef, net->act.x0, op->sc, stop_mask, s);
        launch_net_forward_fused<Tv>(g, net->d, net->act, q, qp, delta, op->sc, stop_mask, s);
    }
    launch_thomas<Tv>(op->tri_view<Tv>(), qp, z, TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials, nullptr,
                      op->sc, s, stop_mask);
}

// One flexible BiCGStab iteration with the learned preconditioner: the recurrences are those
// of the plain iteration; x is updated with exactly the phat, shat that were multiplied by A.
template <typename Tv, typename Tc>
void enqueue_iteration_learned(eg_operator *op, const OpView<Tc> &A, Work<Tv> &w, eg_net *net, const Tc *coef)
{
    hipStream_t s = op->stream;
    const TriView<Tv> T = op->tri_view<Tv>();
    int nr = 0;
    launch_thomas<Tv>(T, nullptr, w.ph, TH_P, w.r, w.p, w.v, w.rh, op->partials, &nr, op->sc, s);
    enqueue_net_stage<Tv, Tc>(op, net, coef, w.p, w.ph, w.qp, nullptr, STOP_DONE);
    launch_spmv<Tv, Tc>(A, w.ph, w.v, w.rh, SP_DOT2, op->partials, &nr, op->sc, STOP_DONE, s);
    launch_finalize(FIN_SIGMA, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
    launch_thomas<Tv>(T, nullptr, w.sh, TH_S, w.r, w.s, w.v, nullptr, op->partials, &nr, op->sc, s);
    launch_finalize(FIN_S, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
    enqueue_net_stage<Tv, Tc>(op, net, coef, w.s, w.sh, w.qp, nullptr, STOP_DONE | STOP_SKIP | STOP_HALF);
    launch_spmv<Tv, Tc>(A, w.sh, w.t, w.s, SP_DOT2, op->partials, &nr, op->sc, STOP_DONE | STOP_SKIP | STOP_HALF, s);
    launch_finalize(FIN_OMEGA, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
    launch_update<Tv>(op->n, w.x, w.ph, w.sh, w.s, w.t, w.r, w.rh, op->partials, &nr, op->sc, s);
    launch_finalize(FIN_END, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 0, s);
}

// Krylov run with the learned preconditioner, checked after every iteration.  Stall rule:
// the best residual has not halved within stall_window iterations, or the residual exceeds
// 1e3 times the best, or the iteration broke down.  On a stall *fallback is set and the run
// returns with the device state mid-run; the caller continues with T^{-1} alone.
template <typename Tv, typename Tc>
int krylov_run_learned(eg_operator *op, const OpView<Tc> &A, Work<Tv> &w, eg_net *net, const Tc *coef,
                       int *fallback)
{
    *fallback = 0;
    int rc;
    if ((rc = sync_scalars(op))) return rc;
    double best = op->h_sc->last_rel, anchor = best;
    int anchor_it = op->h_sc->iter;
    while (!op->h_sc->done) {
        enqueue_iteration_learned<Tv, Tc>(op, A, w, net, coef);
        EG_HIP(hipGetLastError());
        if ((rc = sync_scalars(op))) return rc;
        const Scalars &h = *op->h_sc;
        if (h.done && h.status == 2) {   // breakdown: hand over to the plain preconditioner
            *fallback = 1;
            return 0;
        }
        if (h.done) break;
        const double R = h.last_rel;
        best = std::min(best, R);
        if (R <= 0.5 * anchor) {
            anchor = R;
            anchor_it = h.iter;
        }
        if (h.iter - anchor_it >= op->stall_window || R > 1e3 * best || !std::isfinite(R)) {
            *fallback = 1;
            return 0;
        }
    }
    return 0;
}

// ---- FGMRES ------------------------------------------------------------------------------
template <typename Tv> int ensure_fgm(eg_operator *op)
{
    Fgm<Tv> &F = op->fgm<Tv>();
    int rc;
    if (!op->d_h) {
        if ((rc = dalloc(&op->d_h, 4 * (kMaxGmres + 2)))) return rc;
        if ((rc = dalloc(&op->mpart, (size_t)8192 * kMBlk))) return rc;
        if (hipHostMalloc(reinterpret_cast<void **>(&op->h_h), 4 * (kMaxGmres + 2) * sizeof(double)) != hipSuccess)
            return fail(EG_ENOMEM, "hipHostMalloc failed");
    }
    if (F.m == op->gm_m && F.V) return 0;
    dfree(F.V); dfree(F.Z); dfree(F.W); dfree(F.R); dfree(F.tmp);
    F.m = 0;
    const size_t n = (size_t)op->n, m = (size_t)op->gm_m;
    if ((rc = dalloc(&F.V, (m + 1) * n)) || (rc = dalloc(&F.Z, m * n)) || (rc = dalloc(&F.W, n)) ||
        (rc = dalloc(&F.R, n)) || (rc = dalloc(&F.tmp, n)))
        return rc;
    F.m = op->gm_m;
    return 0;
}

// Right-preconditioned restarted FGMRES(m) for A d = rhs (Saad's flexible variant: the
// preconditioned vectors z_j are kept, so M may change between applications, e.g. the learned
// M).  On entry F.R holds rhs - A d; resid() must recompute it from the current d.  Classical
// Gram-Schmidt with one reorthogonalisation pass; FP64 dot products.  Histories are relative
// to nb.  Stops at |g| / nb <= tol (then checked against the recomputed residual) or maxit.
// With a network the stall rule of the flexible BiCGStab applies to the residual estimates,
// over at least one restart cycle: when the best residual has not halved within
// max(stall_window, m) steps the cycle ends there and the iteration continues with T^{-1}.
template <typename Tv, typename Tc, typename ResidFn>
int fgmres(eg_operator *op, const OpView<Tc> &A, Tv *d, double nb, double tol, int maxit, eg_net *net,
           const Tc *coef, ResidFn resid, int *iters, int *status, int *fallbacks)
{
    int rc;
    if ((rc = ensure_fgm<Tv>(op))) return rc;
    Fgm<Tv> &F = op->fgm<Tv>();
    hipStream_t s = op->stream;
    const long n = op->n;
    const int m = F.m;
    const TriView<Tv> T = op->tri_view<Tv>();
    bool use_net = net != nullptr;
    Tv *qp = nullptr;
    if (use_net) qp = F.tmp;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hij = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    int it = 0, anchor_it = 0;
    *status = 1;
    double anchor = INFINITY;
    bool stalled = false;
    for (;;) {
        // beta = ||R||
        int nr = 0;
        launch_dot<Tv, Tv>(n, F.R, F.R, op->partials, &nr, s);
        launch_finalize(FIN_SUM, op->partials, nr, op->sc, nullptr, op->d_out, 0, 0, s);
        EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, sizeof(double), hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        const double beta = std::sqrt(op->h_out[0]);
        if (beta / nb <= tol || beta == 0.0) { *status = 0; break; }
        if (it >= maxit) break;
        if (!std::isfinite(beta)) { *status = 2; break; }
        if (stalled) {
            use_net = false;
            *fallbacks += 1;
            stalled = false;
        }
        if (beta / nb <= 0.5 * anchor) {
            anchor = beta / nb;
            anchor_it = it;
        }
        // v0 = R / beta
        op->h_h[0] = beta;
        EG_HIP(hipMemcpyAsync(op->d_h + 2 * (kMaxGmres + 1), op->h_h, sizeof(double), hipMemcpyHostToDevice, s));
        launch_vscale<Tv>(n, F.R, F.V, op->d_h + 2 * (kMaxGmres + 1), s);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = -1;
        for (int j = 0; j < m; ++j) {
            Tv *Vj = F.V + (size_t)j * n, *Zj = F.Z + (size_t)j * n;
            if (op->sor_on && !use_net) {
                Tv *xcm = op->sor_x<Tv>(), *qcm = op->sor_q<Tv>();
                launch_thomas_cm<Tv>(T, op->nlon, Vj, xcm, qcm, TH_PLAIN, nullptr, nullptr, nullptr, nullptr,
                                     op->partials, nullptr, nullptr, s);
                launch_sor<Tv, Tc>(A, op->sor_view<Tv, Tc>(), qcm, xcm, op->sor_w<Tv>(), Zj, op->sor_sweeps,
                                   op->sor_omega, nullptr, 0, s);
            } else {
                launch_thomas<Tv>(T, Vj, Zj, TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials, nullptr,
                                  nullptr, s);
            }
            if constexpr (std::is_same_v<Tc, float> || std::is_same_v<Tc, double>)
                if (use_net) enqueue_net_stage<Tv, Tc>(op, net, coef, Vj, Zj, qp, nullptr, 0);
            launch_spmv<Tv, Tc>(A, Zj, F.W, nullptr, SP_PLAIN, op->partials, nullptr, nullptr, 0, s);
            for (int pass = 0; pass < 2; ++pass) {
                double *hp = op->d_h + pass * (kMaxGmres + 1);
                for (int i0 = 0; i0 <= j; i0 += kMBlk)
                    launch_mdot<Tv>(n, F.W, F.V, i0, std::min(kMBlk, j + 1 - i0), op->mpart, hp, s);
                for (int i0 = 0; i0 <= j; i0 += kMBlk) {
                    const bool last = (pass == 1) && (i0 + kMBlk > j);
                    nr = launch_maxpy<Tv>(n, F.W, F.V, i0, std::min(kMBlk, j + 1 - i0), hp, -1.0, last, op->partials, s);
                }
            }
            launch_finalize(FIN_SUM, op->partials, nr, op->sc, nullptr, op->d_out, 0, 0, s);
            EG_HIP(hipMemcpyAsync(op->h_h, op->d_h, 2 * (kMaxGmres + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
            EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, sizeof(double), hipMemcpyDeviceToHost, s));
            EG_HIP(hipGetLastError());
            EG_HIP(hipStreamSynchronize(s));
            for (int i = 0; i <= j; ++i) Hij(i, j) = op->h_h[i] + op->h_h[kMaxGmres + 1 + i];
            const double hn = std::sqrt(op->h_out[0]);
            Hij(j + 1, j) = hn;
            // v_{j+1} = w / h_{j+1,j}
            if (hn > 0.0) {
                op->h_h[0] = hn;
                EG_HIP(hipMemcpyAsync(op->d_h + 2 * (kMaxGmres + 1), op->h_h, sizeof(double), hipMemcpyHostToDevice,
                                      s));
                launch_vscale<Tv>(n, F.W, F.V + (size_t)(j + 1) * n, op->d_h + 2 * (kMaxGmres + 1), s);
            }
            // Givens rotations: apply the previous ones to column j, then annihilate H(j+1, j)
            for (int i = 0; i < j; ++i) {
                const double a = Hij(i, j), b = Hij(i + 1, j);
                Hij(i, j) = cs[i] * a + sn[i] * b;
                Hij(i + 1, j) = -sn[i] * a + cs[i] * b;
            }
            const double a = Hij(j, j), b = Hij(j + 1, j);
            const double rr = std::hypot(a, b);
            cs[j] = rr > 0.0 ? a / rr : 1.0;
            sn[j] = rr > 0.0 ? b / rr : 0.0;
            Hij(j, j) = rr;
            Hij(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            const double R = std::fabs(g[j + 1]) / nb;
            op->hist_pending.push_back(R);
            jend = j;
            if (R <= 0.5 * anchor) {
                anchor = R;
                anchor_it = it;
            }
            if (use_net && (it - anchor_it >= std::max(op->stall_window, m) || !std::isfinite(R))) stalled = true;
            if (R <= tol || it >= maxit || hn == 0.0 || !std::isfinite(hn) || stalled) break;
        }
        // y = H^{-1} g (upper triangular), d += Z y
        for (int i = jend; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k <= jend; ++k) t -= Hij(i, k) * y[k];
            y[i] = Hij(i, i) != 0.0 ? t / Hij(i, i) : 0.0;
        }
        for (int i = 0; i <= jend; ++i) op->h_h[i] = y[i];
        EG_HIP(hipMemcpyAsync(op->d_h, op->h_h, (jend + 1) * sizeof(double), hipMemcpyHostToDevice, s));
        for (int i0 = 0; i0 <= jend; i0 += kMBlk)
            launch_maxpy<Tv>(n, d, F.Z, i0, std::min(kMBlk, jend + 1 - i0), op->d_h, 1.0, 0, op->partials, s);
        resid();
        EG_HIP(hipGetLastError());
    }
    *iters = it;
    return 0;
}

// rr64 = ||b - A x||^2, bb = ||b||^2 into h_out[0..1]; r (may be null) receives b - A x.
template <typename Tout> int true_residual(eg_operator *op, const double *b, const double *x, Tout *r, int *nrows)
{
    launch_residual<Tout>(op->view64(), b, x, r, op->partials, nrows, op->stream);
    launch_finalize(FIN_SUM, op->partials, *nrows, op->sc, nullptr, op->d_out, 0, 0, op->stream);
    EG_HIP(hipGetLastError());
    EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, op->stream));
    EG_HIP(hipStreamSynchronize(op->stream));
    return 0;
}

int check_vectors(eg_operator *op, const double *b, const double *x)
{
    EG_HIP(hipMemsetAsync(op->d_bad, 0, 4 * sizeof(int), op->stream));
    launch_check_finite(op->n, b, op->d_bad, op->stream);
    launch_check_finite(op->n, x, op->d_bad + 1, op->stream);
    int h[4];
    EG_HIP(hipMemcpyAsync(h, op->d_bad, 4 * sizeof(int), hipMemcpyDeviceToHost, op->stream));
    EG_HIP(hipStreamSynchronize(op->stream));
    if (h[0] || h[1])
        return fail(EG_ENONFINITE, std::to_string(h[0]) + " non-finite values in b, " + std::to_string(h[1]) +
                                       " in x");
    return 0;
}

// ---- plain FP64 BiCGStab --------------------------------------------------------------------
int solve_fp64(eg_operator *op, const double *b, double *x, double tol, int maxit, eg_net *net = nullptr)
{
    int rc;
    if ((rc = ensure_work(op, op->w64))) return rc;
    if (net && ((rc = ensure_qp(op, op->w64)) || (rc = ensure_acts(net, op->n, false)) || (rc = ensure_net_static(op))))
        return rc;
    Work<double> &w = op->w64;
    hipStream_t s = op->stream;
    const OpView<double> A = op->view64();
    EG_HIP(hipMemcpyAsync(w.x, x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if ((rc = put_run_params(op, tol, maxit, 0, op->restart_every))) return rc;
    int nr = 0;
    launch_residual<double>(A, b, w.x, w.r, op->partials, &nr, s);
    launch_finalize(FIN_INIT, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 1, s);
    EG_HIP(hipGetLastError());
    if ((rc = sync_scalars(op))) return rc;
    if (op->h_sc->nb2 == 0.0) {
        launch_fill<double>(x, op->n, 0.0, s);
        EG_HIP(hipStreamSynchronize(s));
        op->info.true_rel_residual = 0.0;
        return EG_CONVERGED;
    }
    if ((net ? op->learned_method : op->method) == 1) {
        // restarted FGMRES(m); every cycle ends on the FP64 true residual
        Fgm<double> *F = nullptr;
        if ((rc = ensure_fgm<double>(op))) return rc;
        F = &op->f64;
        const double nb = std::sqrt(op->h_sc->nb2);
        launch_residual<double>(A, b, w.x, F->R, op->partials, &nr, s);
        auto resid = [&]() { launch_residual<double>(A, b, w.x, F->R, op->partials, &nr, s); };
        int its = 0, st = 1, fb = 0;
        if ((rc = fgmres<double, double>(op, A, w.x, nb, tol, maxit, net, op->a64, resid, &its, &st, &fb))) return rc;
        op->info.iterations = its;
        op->info.fallbacks += fb;
        op->hist_count = its;
        EG_HIP(hipMemcpyAsync(x, w.x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
        int n2;
        if ((rc = true_residual<double>(op, b, x, static_cast<double *>(nullptr), &n2))) return rc;
        op->info.true_rel_residual = std::sqrt(op->h_out[0] / op->h_out[1]);
        if (op->info.true_rel_residual <= tol) return EG_CONVERGED;
        return st == 2 ? EG_BREAKDOWN : (its >= maxit ? EG_MAXIT : EG_STALLED);
    }
    int gap = 0, status = EG_CONVERGED;
    bool use_net = net != nullptr;
    for (;;) {
        if (use_net) {
            int fb = 0;
            if ((rc = krylov_run_learned<double, double>(op, A, w, net, op->a64, &fb))) return rc;
            if (fb) {   // stall: continue with T^{-1}, restarted from the true residual
                use_net = false;
                op->info.fallbacks += 1;
                if (op->h_sc->iter >= op->h_sc->maxit) { status = EG_MAXIT; break; }
                launch_residual<double>(A, b, w.x, w.r, op->partials, &nr, s);
                launch_finalize(FIN_TRUE, op->partials, nr, op->sc, nullptr, nullptr, 0, 1, s);
                EG_HIP(hipGetLastError());
                continue;
            }
        } else if ((rc = krylov_run<double, double>(op, A, w))) {
            return rc;
        }
        const Scalars &h = *op->h_sc;
        if (h.status == 4) {   // periodic restart: fresh true residual
            launch_residual<double>(A, b, w.x, w.r, op->partials, &nr, s);
            launch_finalize(FIN_TRUE, op->partials, nr, op->sc, nullptr, nullptr, 0, 1, s);
            EG_HIP(hipGetLastError());
            continue;
        }
        if (h.status == 1) { status = EG_MAXIT; break; }
        if (h.status == 2) { status = EG_BREAKDOWN; break; }
        // converged on the recursive residual: check the true one (residual-gap guard)
        launch_residual<double>(A, b, w.x, w.r, op->partials, &nr, s);
        launch_finalize(FIN_SUM, op->partials, nr, op->sc, nullptr, op->d_out, 0, 0, s);
        EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        const double rel = std::sqrt(op->h_out[0] / op->h_out[1]);
        if (rel <= tol) { status = EG_CONVERGED; break; }
        if (gap >= 3 || h.iter >= h.maxit) { status = (h.iter >= h.maxit) ? EG_MAXIT : EG_STALLED; break; }
        ++gap;
        launch_finalize(FIN_TRUE, op->partials, nr, op->sc, nullptr, nullptr, 0, 1, s);
        EG_HIP(hipGetLastError());
    }
    const Scalars &h = *op->h_sc;
    op->info.iterations = h.iter;
    op->info.restarts = h.restarts;
    op->hist_count = h.iter;
    EG_HIP(hipMemcpyAsync(x, w.x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int n2;
    if ((rc = true_residual<double>(op, b, x, static_cast<double *>(nullptr), &n2))) return rc;
    op->info.true_rel_residual = std::sqrt(op->h_out[0] / op->h_out[1]);
    return status;
}

// ---- FP64 refinement around an FP32 inner BiCGStab ------------------------------------------
template <typename Tc>
int solve_ir(eg_operator *op, const OpView<Tc> &A32, const double *b, double *x, double tol, int maxit,
             eg_net *net = nullptr)
{
    int rc;
    if ((rc = ensure_work(op, op->w32))) return rc;
    if (net && ((rc = ensure_qp(op, op->w32)) || (rc = ensure_acts(net, op->n, false)) || (rc = ensure_net_static(op))))
        return rc;
    bool use_net = net != nullptr;
    Work<float> &w = op->w32;
    hipStream_t s = op->stream;
    if (!op->ir_backup && (rc = dalloc(&op->ir_backup, (size_t)op->n))) return rc;
    int total = 0, outer = 0, status = EG_MAXIT, stalls = 0, restarts = 0;
    double rel_prev = INFINITY;
    bool fallback = false;
    for (;;) {
        int nr = 0;
        if (op->profile) {
            if ((rc = ensure_events(op))) return rc;
            EG_HIP(hipEventRecord(op->ev[10], s));
        }
        launch_residual<float>(op->view64(), b, x, w.r, op->partials, &nr, s);
        if (op->profile) EG_HIP(hipEventRecord(op->ev[11], s));
        launch_finalize(FIN_SUM, op->partials, nr, op->sc, nullptr, op->d_out, 0, 0, s);
        EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        if (op->profile && (rc = add_kernel_time(op, 5, EG_K_RESIDUAL, EG_PREC_FP64))) return rc;
        const double rr = op->h_out[0], bb = op->h_out[1];
        if (bb == 0.0) {
            launch_fill<double>(x, op->n, 0.0, s);
            EG_HIP(hipStreamSynchronize(s));
            op->info.true_rel_residual = 0.0;
            status = EG_CONVERGED;
            break;
        }
        const double rel = std::sqrt(rr / bb);
        op->info.true_rel_residual = rel;
        if (rel <= tol) { status = EG_CONVERGED; break; }
        if (outer > 0 && !(rel < rel_prev)) {
            // the last correction made the residual no smaller (the FP32 inner solve failed,
            // e.g. on a near-singular operator): undo it and finish in FP64
            EG_HIP(hipMemcpyAsync(x, op->ir_backup, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
            op->info.true_rel_residual = rel_prev;
            fallback = true;
            break;
        }
        if (total >= maxit) { status = EG_MAXIT; break; }
        if (outer >= op->max_outer) { status = EG_STALLED; break; }   // the caller's cap on refinement steps
        if (rel > 0.5 * rel_prev) {
            if (++stalls >= (net ? 3 : 2)) { fallback = true; break; }
        } else {
            stalls = 0;
        }
        rel_prev = rel;
        // inner solve  A32 d = r32  to relative tolerance eta (no tighter than this step needs)
        const double eta = std::max(op->eta, 0.25 * tol / rel);
        // a capped inner solve still hands over its correction; the check of the true residual
        // above undoes it if it did not help
        const int inner_cap = std::min(maxit - total, op->inner_maxit);
        if ((rc = put_run_params(op, eta, inner_cap, total, op->restart_every))) return rc;
        launch_finalize(FIN_INIT, op->partials, nr, op->sc, op->d_hist, nullptr, 2, 2, s);
        launch_fill<float>(w.x, op->n, 0.0f, s);
        EG_HIP(hipGetLastError());
        if ((net ? op->learned_method : op->method) == 1) {
            // inner FGMRES on A32 d = r32 (F.R = r32 - A32 d, recomputed after every cycle)
            if ((rc = ensure_fgm<float>(op))) return rc;
            Fgm<float> &F = op->f32;
            EG_HIP(hipMemcpyAsync(F.R, w.r, op->n * sizeof(float), hipMemcpyDeviceToDevice, s));
            const double nb_in = std::sqrt(op->h_out[2]);
            auto resid = [&]() {
                launch_spmv<float, Tc>(A32, w.x, F.tmp, nullptr, SP_PLAIN, op->partials, nullptr, nullptr, 0, s);
                launch_net_diff(op->n, w.r, F.tmp, F.R, s);
            };
            int its = 0, st = 1, fb = 0;
            const Tc *coef = nullptr;
            if constexpr (std::is_same_v<Tc, float>) coef = op->a32;
            if ((rc = fgmres<float, Tc>(op, A32, w.x, nb_in, eta, inner_cap, use_net ? net : nullptr, coef, resid,
                                        &its, &st, &fb)))
                return rc;
            if (fb) {
                use_net = false;
                op->info.fallbacks += fb;
            }
            total += its;
            EG_HIP(hipMemcpyAsync(op->ir_backup, x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
            launch_add_correction(op->n, x, w.x, s);
            EG_HIP(hipGetLastError());
            ++outer;
            continue;
        }
        if constexpr (std::is_same_v<Tc, float>) {
            if (use_net) {
                int fb = 0;
                if ((rc = krylov_run_learned<float, float>(op, A32, w, net, op->a32, &fb))) return rc;
                if (fb) {   // stall: this refinement step ends here, the next ones use T^{-1}
                    use_net = false;
                    op->info.fallbacks += 1;
                }
            } else if ((rc = krylov_run<float, Tc>(op, A32, w))) {
                return rc;
            }
        } else if ((rc = krylov_run<float, Tc>(op, A32, w))) {
            return rc;
        }
        total += op->h_sc->iter;
        restarts += op->h_sc->restarts;
        EG_HIP(hipMemcpyAsync(op->ir_backup, x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_add_correction(op->n, x, w.x, s);
        EG_HIP(hipGetLastError());
        ++outer;
    }
    op->info.iterations = total;
    op->info.outer_steps = outer;
    op->info.restarts = restarts;
    op->hist_count = total;
    if (fallback) {
        // the FP32 refinement cannot go further: continue from x with the FP64 solver (the
        // history then holds the FP64 solve's residuals)
        const eg_info before = op->info;
        if (op->sor_on && (rc = ensure_sor<double>(op))) return rc;
        status = solve_fp64(op, b, x, tol, std::max(1, maxit - total));
        if (status < 0) return status;
        op->info.iterations += before.iterations;
        op->info.outer_steps = before.outer_steps;
        op->info.restarts += before.restarts;
        op->info.fallbacks = before.fallbacks + 1;
    }
    return status;
}

// ---- the paper's mixed-precision BiCGStab (Sec. 3 and Sec. 4) ------------------------------
// FP32 vectors, coefficients and preconditioner; the solution x in FP64, updated every
// iteration; FP64 global sums; a restart from the true residual every restart_every
// iterations (150, the paper's value, when the option is 0).  No refinement: one Krylov run on
// A x = b, halted on the recursive residual and then checked against the FP64 true residual
// (up to three residual-gap restarts, then EG_STALLED: the FP32 recurrence has hit its floor).
int solve_mp(eg_operator *op, const double *b, double *x, double tol, int maxit)
{
    int rc;
    if ((rc = ensure_fp32(op)) || (rc = ensure_work(op, op->w32))) return rc;
    if (!op->mp_x && (rc = dalloc(&op->mp_x, (size_t)op->n))) return rc;
    Work<float> &w = op->w32;
    hipStream_t s = op->stream;
    const OpView<double> A64 = op->view64();
    const OpView<float> A32 = op->view32();
    EG_HIP(hipMemcpyAsync(op->mp_x, x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if ((rc = put_run_params(op, tol, maxit, 0, op->restart_every > 0 ? op->restart_every : 150))) return rc;
    int nr = 0;
    // r = b - A x in FP64, stored in FP32; partials ||r64||^2, ||b||^2, ||r32||^2
    launch_residual<float>(A64, b, op->mp_x, w.r, op->partials, &nr, s);
    launch_finalize(FIN_INIT, op->partials, nr, op->sc, op->d_hist, nullptr, 2, 1, s);
    EG_HIP(hipGetLastError());
    if ((rc = sync_scalars(op))) return rc;
    if (op->h_sc->nb2 == 0.0) {
        launch_fill<double>(x, op->n, 0.0, s);
        EG_HIP(hipStreamSynchronize(s));
        op->info.true_rel_residual = 0.0;
        return EG_CONVERGED;
    }
    struct Guard {
        eg_operator *op;
        ~Guard() { op->mp_active = false; }
    } guard{op};
    op->mp_active = true;
    int gap = 0, status = EG_CONVERGED;
    for (;;) {
        if ((rc = krylov_run<float, float>(op, A32, w))) return rc;
        const Scalars &h = *op->h_sc;
        if (h.status == 4) {   // periodic restart from the true residual
            launch_residual<float>(A64, b, op->mp_x, w.r, op->partials, &nr, s);
            launch_finalize(FIN_TRUE, op->partials, nr, op->sc, nullptr, nullptr, 2, 1, s);
            EG_HIP(hipGetLastError());
            continue;
        }
        if (h.status == 1) { status = EG_MAXIT; break; }
        if (h.status == 2) { status = EG_BREAKDOWN; break; }
        launch_residual<float>(A64, b, op->mp_x, w.r, op->partials, &nr, s);
        launch_finalize(FIN_SUM, op->partials, nr, op->sc, nullptr, op->d_out, 0, 0, s);
        EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        const double rel = std::sqrt(op->h_out[0] / op->h_out[1]);
        if (rel <= tol) { status = EG_CONVERGED; break; }
        if (gap >= 3 || h.iter >= h.maxit) { status = (h.iter >= h.maxit) ? EG_MAXIT : EG_STALLED; break; }
        ++gap;
        launch_finalize(FIN_TRUE, op->partials, nr, op->sc, nullptr, nullptr, 2, 1, s);
        EG_HIP(hipGetLastError());
    }
    const Scalars &h = *op->h_sc;
    op->info.iterations = h.iter;
    op->info.restarts = h.restarts;
    op->hist_count = h.iter;
    EG_HIP(hipMemcpyAsync(x, op->mp_x, op->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int n2;
    if ((rc = true_residual<double>(op, b, x, static_cast<double *>(nullptr), &n2))) return rc;
    op->info.true_rel_residual = std::sqrt(op->h_out[0] / op->h_out[1]);
    return status;
}

// ---- network training pieces ---------------------------------------------------------------
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

double std_normal(uint64_t &s)   // Box-Muller
{
    const double u1 = uniform01(s), u2 = uniform01(s);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// One training pair on the given stream: forward, the loss into *loss_slot (device), and (if
// backward) this pair's per-row partial weight gradients, written into net->d.part for the
// first pair of a batch and added for the others (launch_net_grad sums them into d.grad).
int net_pair_pass(eg_net *net, eg_operator *op, const float *r, const float *e, bool backward, int first,
                  double *loss_slot, hipStream_t s)
{
    int rc;
    if ((rc = ensure_fp32(op)) || (rc = ensure_acts(net, op->n, backward)) || (rc = ensure_train_tmp(net, op->n)))
        return rc;
    const long n = op->n;
    const NetGeo g = geo_of(op);
    const TriView<float> T = op->tri_view32();
    int nr = 0;
    launch_thomas<float>(T, r, net->t_z0, TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials, nullptr, nullptr,
                         s);
    launch_dot2<float>(n, r, r, net->t_z0, net->t_z0, op->partials, &nr, nullptr, 0, s);
    launch_finalize(FIN_NET, op->partials, nr, op->sc, nullptr, nullptr, 0, 0, s);
    launch_net_features<float, float>(g, r, net->t_z0, op->a32, net->act.x0, op->sc, 0, s);
    launch_net_forward_layers(g, net->d, net->act, op->sc, 0, s);
    launch_net_out<float>(g, net->d, net->act, r, net->t_qp, nullptr, op->sc, 0, s);
    launch_thomas<float>(T, net->t_qp, net->t_m, TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials, nullptr,
                         nullptr, s);
    if (net->loss_kind == 1) {
        // residual space: d = A m - r, loss ||d||^2 / ||r||^2, dL/dm = A^T (2 d / ||r||^2)
        launch_spmv<float, float>(op->view32(), net->t_m, net->t_g, nullptr, SP_PLAIN, op->partials, nullptr, nullptr,
                                  0, s);
        launch_net_diff(n, net->t_g, r, net->t_diff, s);
        launch_dot2<float>(n, net->t_diff, net->t_diff, r, r, op->partials, &nr, nullptr, 0, s);
        launch_finalize(FIN_LOSS, op->partials, nr, op->sc, nullptr, loss_slot, 0, 0, s);
        if (backward) {
            launch_net_gseed(n, net->t_g, r, net->t_g, op->sc, s);
            launch_spmv_t(g, op->a32, op->m32, net->t_g, net->t_z0, s);
            launch_thomas_t(T, net->t_z0, net->t_u, s);
            launch_net_backward(g, net->d, net->act, net->t_u, op->sc, first, s);
        }
    } else {
        // error space: loss ||m - e||^2 / ||e||^2, dL/dm = 2 (m - e) / ||e||^2
        launch_net_diff(n, net->t_m, e, net->t_diff, s);
        launch_dot2<float>(n, net->t_diff, net->t_diff, e, e, op->partials, &nr, nullptr, 0, s);
        launch_finalize(FIN_LOSS, op->partials, nr, op->sc, nullptr, loss_slot, 0, 0, s);
        if (backward) {
            launch_net_gseed(n, net->t_m, e, net->t_g, op->sc, s);
            launch_thomas_t(T, net->t_g, net->t_u, s);
            launch_net_backward(g, net->d, net->act, net->t_u, op->sc, first, s);
        }
    }
    EG_HIP(hipGetLastError());
    return 0;
}

int ensure_loss(eg_net *net, long npairs)
{
    if (npairs <= net->loss_cap) return 0;
    dfree(net->d_loss);
    int rc = dalloc(&net->d_loss, (size_t)npairs);
    if (rc) return rc;
    net->loss_cap = npairs;
    return 0;
}

// Settings of eg_train_learned_pc ("key=value,key=value").
struct PcCfg {
    int source = 0;   // 0: iterates of an FP64 solve (eg_harvest), 1: FGMRES basis (eg_harvest_krylov)
    int rhs = 8;
    int pairs = 20;
    int loss = 0;     // 0 error space, 1 residual space
    int batch = 16;
};

int parse_pc_cfg(const char *cfg, PcCfg &c)
{
    if (!cfg) return 0;
    const std::string all(cfg);
    size_t pos = 0;
    while (pos < all.size()) {
        size_t end = all.find(',', pos);
        if (end == std::string::npos) end = all.size();
        const std::string item = all.substr(pos, end - pos);
        pos = end + 1;
        if (item.empty()) continue;
        const size_t eq = item.find('=');
        if (eq == std::string::npos) return fail(EG_EINVAL, "harvest_cfg: '" + item + "' is not key=value");
        const std::string key = item.substr(0, eq), val = item.substr(eq + 1);
        auto as_int = [&](int lo, int hi, int *out) {
            char *endp = nullptr;
            const long v = std::strtol(val.c_str(), &endp, 10);
            if (val.empty() || *endp != '\0' || v < lo || v > hi)
                return fail(EG_EINVAL, "harvest_cfg: " + key + " must be an integer in [" + std::to_string(lo) + ", " +
                                           std::to_string(hi) + "]");
            *out = (int)v;
            return 0;
        };
        int rc = 0;
        if (key == "source") {
            if (val == "iterates") c.source = 0;
            else if (val == "krylov") c.source = 1;
            else return fail(EG_EINVAL, "harvest_cfg: source must be iterates or krylov");
        } else if (key == "loss") {
            if (val == "error") c.loss = 0;
            else if (val == "residual") c.loss = 1;
            else return fail(EG_EINVAL, "harvest_cfg: loss must be error or residual");
        } else if (key == "rhs") {
            rc = as_int(1, 4096, &c.rhs);
        } else if (key == "pairs") {
            rc = as_int(1, kMaxGmres, &c.pairs);
        } else if (key == "batch") {
            rc = as_int(1, 1 << 20, &c.batch);
        } else {
            return fail(EG_EINVAL, "harvest_cfg: unknown key '" + key + "'");
        }
        if (rc) return rc;
    }
    return 0;
}

constexpr long kPcImageBytes = 16 + 4L * kNetParams;   // header + FP32 weights

int check_pairs(eg_operator *const *ops, int nops, const float *r, const float *e, const int *pair_op, int npairs)
{
    if (!ops || nops < 1 || !r || !e || !pair_op || npairs < 1) return fail(EG_EINVAL, "bad training arguments");
    for (int i = 0; i < nops; ++i) {
        if (!ops[i]) return fail(EG_EINVAL, "NULL operator in the list");
        if (ops[i]->n != ops[0]->n) return fail(EG_EINVAL, "all training operators must have the same grid");
    }
    for (int i = 0; i < npairs; ++i)
        if (pair_op[i] < 0 || pair_op[i] >= nops) return fail(EG_EINVAL, "pair_op index out of range");
    return 0;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

const char *eg_last_error(void) { return g_err.c_str(); }

void eg_destroy_operator(eg_operator *op)
{
    if (!op) return;
    (void)hipStreamSynchronize(op->stream);
    dfree(op->a64); dfree(op->m64); dfree(op->tri64);
    dfree(op->a32); dfree(op->m32); dfree(op->tri32);
    for (int i = 0; i < 2; ++i) { dfree(op->aq[i]); dfree(op->qs[i]); }
    dfree(op->harvest_x);
    for (Fgm<double> *F : {&op->f64}) { dfree(F->V); dfree(F->Z); dfree(F->W); dfree(F->R); dfree(F->tmp); }
    for (Fgm<float> *F : {&op->f32}) { dfree(F->V); dfree(F->Z); dfree(F->W); dfree(F->R); dfree(F->tmp); }
    dfree(op->d_h); dfree(op->mpart); dfree(op->sor_ws); dfree(op->mp_x); dfree(op->ir_backup);
    dfree(op->sorf64); dfree(op->sora64); dfree(op->sorf32); dfree(op->sora32); dfree(op->sorq[0]); dfree(op->sorq[1]);
    if (op->h_h) (void)hipHostFree(op->h_h);
    dfree(op->w64.qp);
    dfree(op->w32.qp);
    for (Work<double> *w : {&op->w64}) {
        dfree(w->r); dfree(w->rh); dfree(w->p); dfree(w->ph); dfree(w->v); dfree(w->s); dfree(w->sh);
        dfree(w->t); dfree(w->x);
    }
    for (Work<float> *w : {&op->w32}) {
        dfree(w->r); dfree(w->rh); dfree(w->p); dfree(w->ph); dfree(w->v); dfree(w->s); dfree(w->sh);
        dfree(w->t); dfree(w->x);
    }
    if (op->ev_ready)
        for (hipEvent_t e : op->ev) (void)hipEventDestroy(e);
    for (const IterGraph &g : op->graphs) (void)hipGraphExecDestroy(g.exec);
    if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
    dfree(op->partials); dfree(op->sc); dfree(op->d_out); dfree(op->d_bad); dfree(op->d_hist);
    if (op->h_sc) (void)hipHostFree(op->h_sc);
    if (op->h_out) (void)hipHostFree(op->h_out);
    if (op->own_net) eg_net_destroy(op->own_net);
    dfree(op->net_fs);
    delete op;
}

int eg_create_operator(const double *coeffs, int nlon, int nlat, int nlev, eg_operator **out)
{
    if (!out) return fail(EG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!coeffs) return fail(EG_EINVAL, "coeffs is NULL");
    if (nlon < 3 || nlat < 1 || nlev < 1) return fail(EG_EINVAL, "need nlon >= 3, nlat >= 1, nlev >= 1");
    const long P = (long)nlon * nlat;
    const long n = P * nlev;
    if (n > (1L << 40)) return fail(EG_EINVAL, "grid too large");
    eg_operator *op = new eg_operator();
    op->nlon = nlon; op->nlat = nlat; op->nlev = nlev; op->P = P; op->n = n;
    int rc = 0;
    auto bail = [&](int code) { eg_destroy_operator(op); return code; };
    if ((rc = dalloc(&op->a64, 6 * (size_t)n)) || (rc = dalloc(&op->m64, (size_t)n)) ||
        (rc = dalloc(&op->tri64, 3 * (size_t)n)) ||
        (rc = dalloc(&op->partials, (size_t)partial_rows_needed(nlon, nlat, nlev) * kPartialCols)) ||
        (rc = dalloc(&op->sc, 1)) || (rc = dalloc(&op->d_out, 4)) || (rc = dalloc(&op->d_bad, 4)))
        return bail(rc);
    if (hipHostMalloc(reinterpret_cast<void **>(&op->h_sc), sizeof(Scalars)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&op->h_out), 4 * sizeof(double)) != hipSuccess)
        return bail(fail(EG_ENOMEM, "hipHostMalloc failed"));
    if ((rc = ensure_hist(op, 4096))) return bail(rc);
    int bad[4] = {0, 0, 0, 0};
    if (hipMemsetAsync(op->d_bad, 0, 4 * sizeof(int), op->stream) != hipSuccess) return bail(fail(EG_EHIP, "memset"));
    launch_derive(coeffs, nlon, nlat, nlev, op->a64, op->m64, op->d_bad, op->stream);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(bad, op->d_bad, sizeof(bad), hipMemcpyDeviceToHost, op->stream) != hipSuccess ||
        hipStreamSynchronize(op->stream) != hipSuccess)
        return bail(fail(EG_EHIP, "operator setup kernel failed"));
    if (bad[0] || bad[1] || bad[2] || bad[3]) {
        std::string m = "invalid operator: " + std::to_string(bad[0]) + " non-finite, " + std::to_string(bad[1]) +
                        " negative couplings, " + std::to_string(bad[2]) + " couplings across a boundary, " +
                        std::to_string(bad[3]) + " rows without a positive margin C - sum(a)";
        return bail(fail(EG_EINVAL, m));
    }
    launch_tri_factor<double>(op->a64, op->m64, nlon, nlat, nlev, op->tri64, op->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(op->stream) != hipSuccess)
        return bail(fail(EG_EHIP, "tridiagonal factorisation failed"));
    *out = op;
    return 0;
}

int eg_set_stream(eg_operator *op, void *hip_stream)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    op->stream = static_cast<hipStream_t>(hip_stream);
    return 0;
}

int eg_set_option(eg_operator *op, const char *key, double value)
{
    if (!op || !key) return fail(EG_EINVAL, "NULL argument");
    const std::string k(key);
    if (k == "eta") {
        if (!(value > 0.0 && value < 1.0)) return fail(EG_EINVAL, "eta must be in (0, 1)");
        op->eta = value;
    } else if (k == "restart_every") {
        if (value < 0) return fail(EG_EINVAL, "restart_every must be >= 0");
        op->restart_every = (int)value;
    } else if (k == "max_outer") {
        if (value < 1) return fail(EG_EINVAL, "max_outer must be >= 1");
        op->max_outer = (int)value;
    } else if (k == "inner_maxit") {
        if (value < 1 || value != std::floor(value)) return fail(EG_EINVAL, "inner_maxit must be an integer >= 1");
        op->inner_maxit = (int)std::min(value, 1e9);
    } else if (k == "poll") {
        if (value < 1 || value > 4096) return fail(EG_EINVAL, "poll must be in [1, 4096]");
        op->poll = (int)value;
    } else if (k == "precond") {
        if (value != 0.0 && value != 1.0) return fail(EG_EINVAL, "precond must be 0 (T^-1) or 1 (red-black line SOR)");
        if (value == 1.0 && op->nlon % 2 != 0) return fail(EG_EINVAL, "the red-black line SOR needs an even nlon");
        op->precond = (int)value;
    } else if (k == "sor_sweeps") {
        if (value < 1 || value > 16 || value != std::floor(value)) return fail(EG_EINVAL, "sor_sweeps must be in 1..16");
        op->sor_sweeps = (int)value;
    } else if (k == "sor_omega") {
        if (!(value > 0.0 && value < 2.0)) return fail(EG_EINVAL, "sor_omega must be in (0, 2)");
        op->sor_omega = value;
    } else if (k == "method") {
        if (value != 0.0 && value != 1.0) return fail(EG_EINVAL, "method must be 0 (BiCGStab) or 1 (FGMRES)");
        op->method = (int)value;
    } else if (k == "learned_method") {
        if (value != 0.0 && value != 1.0) return fail(EG_EINVAL, "learned_method must be 0 or 1");
        op->learned_method = (int)value;
    } else if (k == "gmres_m") {
        if (value < 1 || value > kMaxGmres) return fail(EG_EINVAL, "gmres_m must be in [1, 64]");
        op->gm_m = (int)value;
    } else if (k == "profile") {
        op->profile = value != 0.0;
    } else if (k == "graph") {
        if (value != 0.0 && value != 1.0) return fail(EG_EINVAL, "graph must be 0 or 1");
        op->use_graph = (int)value;
    } else if (k == "eps_bd") {
        if (!(value >= 0.0 && value < 1.0)) return fail(EG_EINVAL, "eps_bd must be in [0, 1)");
        op->eps_bd = value;
    } else if (k == "mp_x32") {
        if (value != 0.0 && value != 1.0) return fail(EG_EINVAL, "mp_x32 must be 0 or 1");
        op->mp_x32 = value != 0.0;
    } else if (k == "net_fused") {
        if (value != 0.0 && value != 1.0) return fail(EG_EINVAL, "net_fused must be 0 or 1");
        op->net_fused = (int)value;
    } else if (k == "stall_window") {
        if (value < 1) return fail(EG_EINVAL, "stall_window must be >= 1");
        op->stall_window = (int)value;
    } else {
        return fail(EG_EINVAL, "unknown option '" + k + "'");
    }
    return 0;
}

int eg_get_shape(const eg_operator *op, int *nlon, int *nlat, int *nlev)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    if (nlon) *nlon = op->nlon;
    if (nlat) *nlat = op->nlat;
    if (nlev) *nlev = op->nlev;
    return 0;
}

int eg_solve(eg_operator *op, const double *b, double *x, double tol, int maxit, int mode)
{
    if (!op || !b || !x) return fail(EG_EINVAL, "NULL argument");
    if (!(tol > 0.0) || maxit < 1) return fail(EG_EINVAL, "need tol > 0 and maxit >= 1");
    if (mode < EG_FP64 || mode > EG_FP32_MP) return fail(EG_EINVAL, "unknown mode");
    const bool learned = (mode == EG_LEARNED_FP64 || mode == EG_LEARNED_FP32_IR);
    if (learned && !op->net)
        return fail(EG_ENOPC, "no learned preconditioner is attached to this operator (eg_attach_learned_pc)");
    const auto t0 = std::chrono::steady_clock::now();
    op->info = eg_info{};
    op->hist_count = 0;
    op->hist_pending.clear();
    int rc;
    // the line SOR is on for this solve only, whichever way it returns
    struct SorScope {
        eg_operator *op;
        ~SorScope() { op->sor_on = false; }
    } sor_scope{op};
    op->sor_on = (op->precond == 1) && !learned;
    if (op->sor_on) {
        if (mode == EG_FP64) rc = ensure_sor<double>(op);
        else if (mode == EG_FP32_IR || mode == EG_FP32_MP) rc = ensure_sor<float>(op);
        else if (mode == EG_FP32_IR_BF16) rc = ensure_sor<bf16_t>(op);
        else rc = ensure_sor<fp16_t>(op);
        if (rc) return rc;
    }
    if ((rc = check_vectors(op, b, x))) return rc;
    if ((rc = ensure_hist(op, std::min(maxit, 1 << 22)))) return rc;
    int status;
    switch (mode) {
    case EG_FP64:
        status = solve_fp64(op, b, x, tol, maxit);
        break;
    case EG_FP32_IR:
        if ((rc = ensure_fp32(op))) return rc;
        status = solve_ir<float>(op, op->view32(), b, x, tol, maxit);
        break;
    case EG_FP32_IR_BF16:
        if ((rc = ensure_quant(op, PBF16))) return rc;
        status = solve_ir<bf16_t>(op, op->viewq<bf16_t>(0), b, x, tol, maxit);
        break;
    case EG_FP32_IR_FP16:
        if ((rc = ensure_quant(op, PFP16))) return rc;
        status = solve_ir<fp16_t>(op, op->viewq<fp16_t>(1), b, x, tol, maxit);
        break;
    case EG_LEARNED_FP64:
        status = solve_fp64(op, b, x, tol, maxit, op->net);
        break;
    case EG_FP32_MP:
        status = solve_mp(op, b, x, tol, maxit);
        break;
    default:
        if ((rc = ensure_fp32(op))) return rc;
        status = solve_ir<float>(op, op->view32(), b, x, tol, maxit, op->net);
        break;
    }
    if (status < 0) return status;
    // history to the host
    if (!op->hist_pending.empty()) {
        op->hist_host = op->hist_pending;
        op->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return status;
    }
    const int cnt = std::min(op->hist_count, op->hist_cap);
    op->hist_host.assign(cnt, 0.0);
    if (cnt > 0) {
        EG_HIP(hipMemcpyAsync(op->hist_host.data(), op->d_hist, cnt * sizeof(double), hipMemcpyDeviceToHost,
                              op->stream));
        EG_HIP(hipStreamSynchronize(op->stream));
    }
    op->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

int eg_kernel_stats(const eg_operator *op, int kernel, int prec, long *launches, double *total_ms)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    if (kernel < 0 || kernel >= EG_K_COUNT || prec < 0 || prec > 3) return fail(EG_EINVAL, "bad kernel or prec");
    if (launches) *launches = op->kcnt[kernel][prec];
    if (total_ms) *total_ms = op->kms[kernel][prec];
    return 0;
}

int eg_reset_kernel_stats(eg_operator *op)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    std::memset(op->kms, 0, sizeof(op->kms));
    std::memset(op->kcnt, 0, sizeof(op->kcnt));
    return 0;
}

int eg_get_info(const eg_operator *op, eg_info *info)
{
    if (!op || !info) return fail(EG_EINVAL, "NULL argument");
    *info = op->info;
    return 0;
}

int eg_residual_history(const eg_operator *op, double *host_buf, int cap)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    const int cnt = (int)op->hist_host.size();
    if (host_buf && cap > 0) std::memcpy(host_buf, op->hist_host.data(), std::min(cap, cnt) * sizeof(double));
    return cnt;
}

int eg_apply(eg_operator *op, const void *x, void *y, int prec)
{
    if (!op || !x || !y) return fail(EG_EINVAL, "NULL argument");
    int rc;
    switch (prec) {
    case EG_PREC_FP64:
        launch_spmv<double, double>(op->view64(), static_cast<const double *>(x), static_cast<double *>(y), nullptr,
                                    SP_PLAIN, op->partials, nullptr, nullptr, 0, op->stream);
        break;
    case EG_PREC_FP32:
        if ((rc = ensure_fp32(op))) return rc;
        launch_spmv<float, float>(op->view32(), static_cast<const float *>(x), static_cast<float *>(y), nullptr,
                                  SP_PLAIN, op->partials, nullptr, nullptr, 0, op->stream);
        break;
    case EG_PREC_BF16:
        if ((rc = ensure_quant(op, PBF16))) return rc;
        launch_spmv<float, bf16_t>(op->viewq<bf16_t>(0), static_cast<const float *>(x), static_cast<float *>(y),
                                   nullptr, SP_PLAIN, op->partials, nullptr, nullptr, 0, op->stream);
        break;
    case EG_PREC_FP16:
        if ((rc = ensure_quant(op, PFP16))) return rc;
        launch_spmv<float, fp16_t>(op->viewq<fp16_t>(1), static_cast<const float *>(x), static_cast<float *>(y),
                                   nullptr, SP_PLAIN, op->partials, nullptr, nullptr, 0, op->stream);
        break;
    default:
        return fail(EG_EINVAL, "unknown precision");
    }
    EG_HIP(hipGetLastError());
    EG_HIP(hipStreamSynchronize(op->stream));
    return 0;
}

int eg_apply_precond(eg_operator *op, const void *q, void *z, int prec)
{
    if (!op || !q || !z) return fail(EG_EINVAL, "NULL argument");
    if (prec < EG_PREC_FP64 || prec > EG_PREC_FP16) return fail(EG_EINVAL, "unknown precision");
    int rc;
    const bool sor = op->precond == 1;
    hipStream_t s = op->stream;
    if (prec == EG_PREC_FP64) {
        const double *qd = static_cast<const double *>(q);
        double *zd = static_cast<double *>(z);
        if (sor) {
            if ((rc = ensure_sor<double>(op))) return rc;
            launch_thomas_cm<double>(op->tri_view64(), op->nlon, qd, op->sor_x<double>(), op->sor_q<double>(),
                                     TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials, nullptr, nullptr, s);
            launch_sor<double, double>(op->view64(), op->sor_view<double, double>(), op->sor_q<double>(),
                                       op->sor_x<double>(), op->sor_w<double>(), zd, op->sor_sweeps, op->sor_omega,
                                       nullptr, 0, s);
        } else {
            launch_thomas<double>(op->tri_view64(), qd, zd, TH_PLAIN, nullptr, nullptr, nullptr, nullptr,
                                  op->partials, nullptr, nullptr, s);
        }
    } else {
        // every lower-precision set uses the FP32 rounding of the FP64 factors
        if ((rc = ensure_fp32(op))) return rc;
        const float *qf = static_cast<const float *>(q);
        float *zf = static_cast<float *>(z);
        if (sor) {
            if (prec == EG_PREC_FP32) rc = ensure_sor<float>(op);
            else if (prec == EG_PREC_BF16) rc = ensure_sor<bf16_t>(op);
            else rc = ensure_sor<fp16_t>(op);
            if (rc) return rc;
            float *xcm = op->sor_x<float>(), *qcm = op->sor_q<float>(), *wsc = op->sor_w<float>();
            launch_thomas_cm<float>(op->tri_view32(), op->nlon, qf, xcm, qcm, TH_PLAIN, nullptr, nullptr, nullptr,
                                    nullptr, op->partials, nullptr, nullptr, s);
            if (prec == EG_PREC_FP32)
                launch_sor<float, float>(op->view32(), op->sor_view<float, float>(), qcm, xcm, wsc, zf,
                                         op->sor_sweeps, op->sor_omega, nullptr, 0, s);
            else if (prec == EG_PREC_BF16)
                launch_sor<float, bf16_t>(op->viewq<bf16_t>(0), op->sor_view<float, bf16_t>(), qcm, xcm, wsc, zf,
                                          op->sor_sweeps, op->sor_omega, nullptr, 0, s);
            else
                launch_sor<float, fp16_t>(op->viewq<fp16_t>(1), op->sor_view<float, fp16_t>(), qcm, xcm, wsc, zf,
                                          op->sor_sweeps, op->sor_omega, nullptr, 0, s);
        } else {
            launch_thomas<float>(op->tri_view32(), qf, zf, TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials,
                                 nullptr, nullptr, s);
        }
    }
    EG_HIP(hipGetLastError());
    EG_HIP(hipStreamSynchronize(op->stream));
    return 0;
}

int eg_residual(eg_operator *op, const double *b, const double *x, double *r, double *rel_host)
{
    if (!op || !b || !x) return fail(EG_EINVAL, "NULL argument");
    int nr, rc;
    if ((rc = true_residual<double>(op, b, x, r, &nr))) return rc;
    if (rel_host) *rel_host = op->h_out[1] > 0.0 ? std::sqrt(op->h_out[0] / op->h_out[1]) : 0.0;
    return 0;
}

int eg_dot(eg_operator *op, const void *a, const void *b, long n, int prec, double *out_host)
{
    if (!op || !a || !b || !out_host || n < 0) return fail(EG_EINVAL, "bad argument");
    int nr = 0;
    if (prec == EG_PREC_FP64)
        launch_dot<double, double>(n, static_cast<const double *>(a), static_cast<const double *>(b), op->partials, &nr,
                                   op->stream);
    else
        launch_dot<float, float>(n, static_cast<const float *>(a), static_cast<const float *>(b), op->partials, &nr,
                                 op->stream);
    launch_finalize(FIN_SUM, op->partials, nr, op->sc, nullptr, op->d_out, 0, 0, op->stream);
    EG_HIP(hipGetLastError());
    EG_HIP(hipMemcpyAsync(op->h_out, op->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, op->stream));
    EG_HIP(hipStreamSynchronize(op->stream));
    *out_host = op->h_out[0];
    return 0;
}

int eg_dot_noalloc(const void *a, const void *b, long n, int prec, void *hip_stream, double *out_host)
{
    if (!a || !b || !out_host) return fail(EG_EINVAL, "NULL argument");
    if (n < 0 || n > kNoAllocMaxN) return fail(EG_EINVAL, "n must be in [0, 2^40]");
    if (prec < EG_PREC_FP64 || prec > EG_PREC_FP16) return fail(EG_EINVAL, "unknown precision");
    double *ws = nullptr;
    int rc;
    if ((rc = scratch_ptr(&ws))) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int nr = 0;
    // the same kernels as eg_dot: partial rows (every row the sum reads is written first), then
    // the fixed-order sum into the four doubles after them
    if (prec == EG_PREC_FP64)
        launch_dot<double, double>(n, static_cast<const double *>(a), static_cast<const double *>(b), ws, &nr, s);
    else
        launch_dot<float, float>(n, static_cast<const float *>(a), static_cast<const float *>(b), ws, &nr, s);
    if (nr > kNoAllocRows) return fail(EG_EINVAL, "internal: more partial rows than the static array holds");
    double *res = ws + (size_t)kNoAllocRows * kPartialCols;
    launch_finalize(FIN_SUM, ws, nr, nullptr, nullptr, res, 0, 0, s);
    EG_HIP(hipGetLastError());
    EG_HIP(hipMemcpyAsync(out_host, res, sizeof(double), hipMemcpyDeviceToHost, s));
    EG_HIP(hipStreamSynchronize(s));
    return 0;
}

// ---------------------------------------------------------------------------------------------
// learned preconditioner
// ---------------------------------------------------------------------------------------------
void eg_net_destroy(eg_net *net)
{
    if (!net) return;
    (void)hipDeviceSynchronize();
    NetDev &d = net->d;
    dfree(d.theta); dfree(d.grad); dfree(d.adam_m); dfree(d.adam_v); dfree(d.part);
    dfree(d.w1f); dfree(d.w2f); dfree(d.w3f); dfree(d.w2b); dfree(d.w3b); dfree(d.w4);
    NetActs &a = net->act;
    dfree(a.x0); dfree(a.a1); dfree(a.a2); dfree(a.a3); dfree(a.d1); dfree(a.d2);
    dfree(net->t_z0); dfree(net->t_qp); dfree(net->t_m); dfree(net->t_diff); dfree(net->t_g); dfree(net->t_u);
    dfree(net->d_loss);
    delete net;
}

int eg_net_set_weights(eg_net *net, const float *host, long count)
{
    if (!net || !host) return fail(EG_EINVAL, "NULL argument");
    if (count != kNetParams) return fail(EG_EINVAL, "expected " + std::to_string(kNetParams) + " weights");
    EG_HIP(hipMemcpy(net->d.theta, host, kNetParams * sizeof(float), hipMemcpyHostToDevice));
    EG_HIP(hipMemset(net->d.adam_m, 0, kNetParams * sizeof(float)));
    EG_HIP(hipMemset(net->d.adam_v, 0, kNetParams * sizeof(float)));
    net->step = 0;
    launch_net_refresh(net->d, nullptr);
    EG_HIP(hipGetLastError());
    EG_HIP(hipDeviceSynchronize());
    return 0;
}

int eg_net_get_weights(const eg_net *net, float *host, long cap)
{
    if (!net) return fail(EG_EINVAL, "NULL net");
    if (host && cap >= kNetParams) {
        EG_HIP(hipDeviceSynchronize());
        EG_HIP(hipMemcpy(host, net->d.theta, kNetParams * sizeof(float), hipMemcpyDeviceToHost));
    }
    return kNetParams;
}

int eg_net_create(unsigned long long seed, eg_net **out)
{
    if (!out) return fail(EG_EINVAL, "out is NULL");
    *out = nullptr;
    eg_net *net = new eg_net();
    NetDev &d = net->d;
    int rc;
    if ((rc = dalloc(&d.theta, kNetParams)) || (rc = dalloc(&d.grad, kNetParams)) ||
        (rc = dalloc(&d.adam_m, kNetParams)) || (rc = dalloc(&d.adam_v, kNetParams)) ||
        (rc = dalloc(&d.part, (size_t)kNetPartRows * kNetParams)) || (rc = dalloc(&d.w1f, 32 * 32)) ||
        (rc = dalloc(&d.w2f, 9 * 1024)) || (rc = dalloc(&d.w3f, 5 * 1024)) || (rc = dalloc(&d.w2b, 9 * 1024)) ||
        (rc = dalloc(&d.w3b, 5 * 1024)) || (rc = dalloc(&d.w4, 160))) {
        eg_net_destroy(net);
        return rc;
    }
    if (hipMemset(d.w1f, 0, 32 * 32 * sizeof(uint16_t)) != hipSuccess) {
        eg_net_destroy(net);
        return fail(EG_EHIP, "memset");
    }
    // He-normal weights (splitmix64 + Box-Muller), zero biases, zero output layer: M = T^{-1}
    std::vector<float> th(kNetParams, 0.f);
    uint64_t st = seed;
    auto fill = [&](int lo, int hi, double sd) {
        for (int i = lo; i < hi; ++i) th[i] = static_cast<float>(sd * std_normal(st));
    };
    fill(kNetOffW1, kNetOffB1, std::sqrt(2.0 / 20.0));
    fill(kNetOffW2, kNetOffB2, std::sqrt(2.0 / 288.0));
    fill(kNetOffW3, kNetOffB3, std::sqrt(2.0 / 160.0));
    if ((rc = eg_net_set_weights(net, th.data(), kNetParams))) {
        eg_net_destroy(net);
        return rc;
    }
    *out = net;
    return 0;
}

int eg_net_set_loss(eg_net *net, int kind)
{
    if (!net || (kind != 0 && kind != 1)) return fail(EG_EINVAL, "loss kind must be 0 or 1");
    net->loss_kind = kind;
    return 0;
}

int eg_attach_learned_pc(eg_operator *op, eg_net *net)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    op->net = net;
    return 0;
}

int eg_net_apply(eg_operator *op, eg_net *net, const float *q, float *z, float *delta)
{
    if (!op || !net || !q || !z) return fail(EG_EINVAL, "NULL argument");
    int rc;
    if ((rc = ensure_fp32(op)) || (rc = ensure_acts(net, op->n, false)) || (rc = ensure_train_tmp(net, op->n)) ||
        (rc = ensure_net_static(op)))
        return rc;
    hipStream_t s = op->stream;
    launch_thomas<float>(op->tri_view32(), q, z, TH_PLAIN, nullptr, nullptr, nullptr, nullptr, op->partials, nullptr,
                         nullptr, s);
    enqueue_net_stage<float, float>(op, net, op->a32, q, z, net->t_qp, delta, 0);
    EG_HIP(hipGetLastError());
    EG_HIP(hipStreamSynchronize(s));
    return 0;
}

int eg_net_loss_grad(eg_operator *op, eg_net *net, const float *r, const float *e, double *loss_host,
                     float *grad_host)
{
    if (!op || !net || !r || !e) return fail(EG_EINVAL, "NULL argument");
    int rc;
    if ((rc = ensure_loss(net, 1))) return rc;
    if ((rc = net_pair_pass(net, op, r, e, true, 1, net->d_loss, op->stream))) return rc;
    launch_net_grad(net->d, 1.f, op->stream);
    EG_HIP(hipGetLastError());
    EG_HIP(hipStreamSynchronize(op->stream));
    if (loss_host) EG_HIP(hipMemcpy(loss_host, net->d_loss, sizeof(double), hipMemcpyDeviceToHost));
    if (grad_host) EG_HIP(hipMemcpy(grad_host, net->d.grad, kNetParams * sizeof(float), hipMemcpyDeviceToHost));
    return 0;
}

int eg_harvest(eg_operator *op, const double *b, int nsnap, float *r_out, float *e_out)
{
    if (!op || !b || !r_out || !e_out || nsnap < 1) return fail(EG_EINVAL, "bad argument");
    int rc;
    op->sor_on = false;   // the harvests use the tridiagonal preconditioner
    if ((rc = check_vectors(op, b, b))) return rc;
    if (!op->harvest_x && (rc = dalloc(&op->harvest_x, (size_t)op->n))) return rc;
    if ((rc = ensure_hist(op, 20000))) return rc;
    hipStream_t s = op->stream;
    // reference solution (as tight as FP64 allows)
    launch_fill<double>(op->harvest_x, op->n, 0.0, s);
    const int st = solve_fp64(op, b, op->harvest_x, 1e-12, 20000);
    if (st < 0) return st;
    // iterates of a fresh solve from x0 = 0, one snapshot after every iteration
    Work<double> &w = op->w64;
    const OpView<double> A = op->view64();
    launch_fill<double>(w.x, op->n, 0.0, s);
    if ((rc = put_run_params(op, 1e-300, std::max(nsnap - 1, 1), 0, 0))) return rc;
    int nr = 0;
    launch_residual<double>(A, b, w.x, w.r, op->partials, &nr, s);
    launch_finalize(FIN_INIT, op->partials, nr, op->sc, op->d_hist, nullptr, 0, 1, s);
    int count = 0;
    for (int i = 0; i < nsnap; ++i) {
        if (i > 0) {   // snapshot 0 is the initial guess x0 = 0 (r_0 = b, e_0 = x*)
            if ((rc = sync_scalars(op))) return rc;
            if (op->h_sc->done) break;
            enqueue_iteration<double, double>(op, A, w, nullptr);
        }
        launch_residual<float>(A, b, w.x, r_out + (size_t)i * op->n, op->partials, &nr, s);
        launch_sub_to_f32(op->n, op->harvest_x, w.x, e_out + (size_t)i * op->n, s);
        EG_HIP(hipGetLastError());
        ++count;
    }
    EG_HIP(hipStreamSynchronize(s));
    return count;
}

int eg_harvest_krylov(eg_operator *op, const double *b, int nvec, float *r_out, float *e_out)
{
    if (!op || !b || !r_out || nvec < 1 || nvec > kMaxGmres) return fail(EG_EINVAL, "bad argument");
    int rc;
    op->sor_on = false;   // the harvests use the tridiagonal preconditioner
    if ((rc = check_vectors(op, b, b))) return rc;
    if ((rc = ensure_work(op, op->w64))) return rc;
    if (!op->harvest_x && (rc = dalloc(&op->harvest_x, (size_t)op->n))) return rc;
    if ((rc = ensure_hist(op, 20000))) return rc;
    // one FGMRES(nvec) cycle with M = T^{-1} from x0 = 0; its basis v_0 .. v_{nvec-1} are the
    // vectors the preconditioner is applied to
    struct Restore {
        eg_operator *op;
        int m, method;
        ~Restore() { op->gm_m = m; op->method = method; op->hist_pending.clear(); }
    } restore{op, op->gm_m, op->method};
    op->gm_m = nvec;
    if ((rc = ensure_fgm<double>(op))) return rc;
    Fgm<double> &F = op->f64;
    Work<double> &w = op->w64;
    hipStream_t s = op->stream;
    const OpView<double> A = op->view64();
    const long n = op->n;
    launch_fill<double>(w.x, n, 0.0, s);
    EG_HIP(hipMemcpyAsync(F.R, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    int nr = 0;
    auto resid = [&]() { launch_residual<double>(A, b, w.x, F.R, op->partials, &nr, s); };
    int its = 0, st = 1, fb = 0;
    if ((rc = fgmres<double, double>(op, A, w.x, 1.0, 0.0, nvec, nullptr, op->a64, resid, &its, &st, &fb)))
        return rc;
    // errors e_j = A^{-1} v_j from tight FP64 BiCGStab solves (the basis is not touched by them)
    op->method = 0;
    for (int j = 0; j < its; ++j) {
        const double *vj = F.V + (size_t)j * n;
        launch_cast_f32(n, vj, r_out + (size_t)j * n, s);
        EG_HIP(hipGetLastError());
        if (!e_out) continue;
        launch_fill<double>(op->harvest_x, n, 0.0, s);
        const int sst = solve_fp64(op, vj, op->harvest_x, 1e-10, 20000);
        if (sst < 0) return sst;
        launch_cast_f32(n, op->harvest_x, e_out + (size_t)j * n, s);
        EG_HIP(hipGetLastError());
    }
    EG_HIP(hipStreamSynchronize(s));
    return its;
}

int eg_net_train(eg_net *net, eg_operator *const *ops, int nops, const float *r, const float *e, const int *pair_op,
                 int npairs, int epochs, int batch, double lr, unsigned long long seed, double *loss_hist)
{
    if (!net || epochs < 0 || batch < 1 || !(lr > 0.0)) return fail(EG_EINVAL, "bad training arguments");
    int rc;
    if ((rc = check_pairs(ops, nops, r, e, pair_op, npairs)) || (rc = ensure_loss(net, npairs))) return rc;
    hipStream_t s = ops[0]->stream;
    const size_t n = (size_t)ops[0]->n;
    std::vector<int> order(npairs);
    std::vector<double> losses(npairs);
    for (int ep = 0; ep < epochs; ++ep) {
        for (int i = 0; i < npairs; ++i) order[i] = i;
        uint64_t st = seed * 1000003ull + (uint64_t)ep;
        for (int i = npairs - 1; i > 0; --i) std::swap(order[i], order[splitmix64(st) % (uint64_t)(i + 1)]);
        for (int b0 = 0; b0 < npairs; b0 += batch) {
            const int b1 = std::min(npairs, b0 + batch);
            const float scale = 1.f / (float)(b1 - b0);
            for (int k = b0; k < b1; ++k) {
                const int pi = order[k];
                if ((rc = net_pair_pass(net, ops[pair_op[pi]], r + (size_t)pi * n, e + (size_t)pi * n, true, k == b0,
                                        net->d_loss + k, s)))
                    return rc;
            }
            launch_net_grad(net->d, scale, s);
            net->step += 1;
            launch_net_adam(net->d, (float)lr, net->step, s);
            EG_HIP(hipGetLastError());
        }
        EG_HIP(hipMemcpyAsync(losses.data(), net->d_loss, npairs * sizeof(double), hipMemcpyDeviceToHost, s));
        EG_HIP(hipStreamSynchronize(s));
        double m = 0.0;
        for (double v : losses) m += v;
        if (loss_hist) loss_hist[ep] = m / npairs;
    }
    return 0;
}

int eg_get_learned_pc(eg_operator *op, eg_net **out)
{
    if (!op || !out) return fail(EG_EINVAL, "NULL argument");
    *out = op->net;
    return op->net ? 0 : fail(EG_ENOPC, "the operator has no learned preconditioner");
}

int eg_train_learned_pc(eg_operator *op, const char *harvest_cfg, int epochs, double lr, unsigned seed)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    if (epochs < 0 || !(lr > 0.0)) return fail(EG_EINVAL, "need epochs >= 0 and lr > 0");
    PcCfg c;
    int rc;
    if ((rc = parse_pc_cfg(harvest_cfg, c))) return rc;
    if (!op->own_net) {
        eg_net *net = nullptr;
        if ((rc = eg_net_create(seed, &net))) return rc;
        op->own_net = net;
    }
    eg_net *net = op->own_net;
    net->loss_kind = c.loss;
    // the pairs live only for this call
    struct Tmp {
        float *r = nullptr, *e = nullptr;
        double *b = nullptr;
        ~Tmp() { dfree(r); dfree(e); dfree(b); }
    } t;
    const size_t n = (size_t)op->n, cap = (size_t)c.rhs * c.pairs;
    if ((rc = dalloc(&t.r, cap * n)) || (rc = dalloc(&t.e, cap * n)) || (rc = dalloc(&t.b, n))) return rc;
    std::vector<double> hb(n);
    long np = 0;
    for (int k = 0; k < c.rhs; ++k) {
        uint64_t st = (uint64_t)seed * 0x9E3779B97F4A7C15ull + 0x51ED270Bull * (uint64_t)(k + 1);
        for (size_t i = 0; i < n; ++i) hb[i] = std_normal(st);
        EG_HIP(hipMemcpyAsync(t.b, hb.data(), n * sizeof(double), hipMemcpyHostToDevice, op->stream));
        EG_HIP(hipStreamSynchronize(op->stream));
        const int cnt = c.source == 0 ? eg_harvest(op, t.b, c.pairs, t.r + (size_t)np * n, t.e + (size_t)np * n)
                                      : eg_harvest_krylov(op, t.b, c.pairs, t.r + (size_t)np * n, t.e + (size_t)np * n);
        if (cnt < 0) return cnt;
        np += cnt;
    }
    if (np < 1) return fail(EG_EINVAL, "the harvest produced no pairs");
    std::vector<int> owner((size_t)np, 0);
    eg_operator *ops[1] = {op};
    if ((rc = eg_net_train(net, ops, 1, t.r, t.e, owner.data(), (int)np, epochs, c.batch, lr, seed, nullptr)))
        return rc;
    op->net = net;
    return 0;
}

int eg_save_learned_pc(const eg_operator *op, void *weights, long cap)
{
    if (!op) return fail(EG_EINVAL, "op is NULL");
    if (!op->net) return fail(EG_ENOPC, "the operator has no learned preconditioner");
    if (!weights) return (int)kPcImageBytes;
    if (cap < kPcImageBytes) return fail(EG_EINVAL, "need " + std::to_string(kPcImageBytes) + " bytes");
    std::vector<float> w(kNetParams);
    int rc = eg_net_get_weights(op->net, w.data(), kNetParams);
    if (rc < 0) return rc;
    const int32_t hdr[3] = {1, kNetParams, 0};
    unsigned char *out = static_cast<unsigned char *>(weights);
    std::memcpy(out, "EGPC", 4);
    std::memcpy(out + 4, hdr, sizeof(hdr));
    std::memcpy(out + 16, w.data(), 4 * (size_t)kNetParams);
    return (int)kPcImageBytes;
}

int eg_load_learned_pc(eg_operator *op, const void *weights, long nbytes)
{
    if (!op || !weights) return fail(EG_EINVAL, "NULL argument");
    if (nbytes != kPcImageBytes) return fail(EG_EINVAL, "a learned-preconditioner image has " +
                                                            std::to_string(kPcImageBytes) + " bytes");
    const unsigned char *in = static_cast<const unsigned char *>(weights);
    int32_t hdr[3];
    std::memcpy(hdr, in + 4, sizeof(hdr));
    if (std::memcmp(in, "EGPC", 4) != 0 || hdr[0] != 1 || hdr[1] != kNetParams || hdr[2] != 0)
        return fail(EG_EINVAL, "not a learned-preconditioner image (header EGPC, version 1, 15233 weights)");
    std::vector<float> w(kNetParams);
    std::memcpy(w.data(), in + 16, 4 * (size_t)kNetParams);
    for (float v : w)
        if (!std::isfinite(v)) return fail(EG_EINVAL, "the image holds non-finite weights");
    int rc;
    if (!op->own_net) {
        eg_net *net = nullptr;
        if ((rc = eg_net_create(0, &net))) return rc;
        op->own_net = net;
    }
    if ((rc = eg_net_set_weights(op->own_net, w.data(), kNetParams))) return rc;
    op->net = op->own_net;
    return 0;
}

int eg_net_eval(eg_net *net, eg_operator *const *ops, int nops, const float *r, const float *e, const int *pair_op,
                int npairs, double *mean_loss)
{
    if (!net || !mean_loss) return fail(EG_EINVAL, "NULL argument");
    int rc;
    if ((rc = check_pairs(ops, nops, r, e, pair_op, npairs)) || (rc = ensure_loss(net, npairs))) return rc;
    hipStream_t s = ops[0]->stream;
    const size_t n = (size_t)ops[0]->n;
    for (int i = 0; i < npairs; ++i)
        if ((rc = net_pair_pass(net, ops[pair_op[i]], r + i * n, e + i * n, false, 1, net->d_loss + i, s)))
            return rc;
    std::vector<double> losses(npairs);
    EG_HIP(hipMemcpyAsync(losses.data(), net->d_loss, npairs * sizeof(double), hipMemcpyDeviceToHost, s));
    EG_HIP(hipStreamSynchronize(s));
    double m = 0.0;
    for (double v : losses) m += v;
    *mean_loss = m / npairs;
    return 0;
}

}  // extern "C"
