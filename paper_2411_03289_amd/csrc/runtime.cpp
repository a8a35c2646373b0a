// Host runtime of the GP-MPPI library: argument validation, context and
// device buffers, GP build orchestration, kernel launches and the closed loop.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "kernels.hpp"

using namespace gpmppi;

namespace {

thread_local std::string g_last_error;

gpmppi_status fail(gpmppi_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(GPMPPI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

bool is_fin(double x) { return std::isfinite(x); }

// Captures one closed-loop step (enqueue, given the capture stream) into a HIP
// graph on a private stream that first waits for the work already queued on st,
// replays it n times, and makes st wait for the replays.  The stream, event,
// graph and executable it creates are released on every return path.
template <class Enqueue>
gpmppi_status replay_captured(hipStream_t st, int n, Enqueue &&enqueue) {
    struct Owned {
        hipStream_t cap = nullptr;
        hipEvent_t ready = nullptr;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool capturing = false;
        ~Owned() {
            if (capturing) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(cap, &g);
                if (g) (void)hipGraphDestroy(g);
            }
            if (cap) (void)hipStreamSynchronize(cap);
            if (exec) (void)hipGraphExecDestroy(exec);
            if (graph) (void)hipGraphDestroy(graph);
            if (ready) (void)hipEventDestroy(ready);
            if (cap) (void)hipStreamDestroy(cap);
        }
    } o;
    HIP_TRY(hipStreamCreateWithFlags(&o.cap, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&o.ready, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(o.ready, st));
    HIP_TRY(hipStreamWaitEvent(o.cap, o.ready, 0));
    HIP_TRY(hipStreamBeginCapture(o.cap, hipStreamCaptureModeThreadLocal));
    o.capturing = true;
    const gpmppi_status s = enqueue(o.cap);
    o.capturing = false;
    const hipError_t ce = hipStreamEndCapture(o.cap, &o.graph);
    if (s != GPMPPI_OK) return s;
    if (ce != hipSuccess) return fail(GPMPPI_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
    HIP_TRY(hipGraphInstantiate(&o.exec, o.graph, nullptr, nullptr, 0));
    for (int t = 0; t < n; ++t) HIP_TRY(hipGraphLaunch(o.exec, o.cap));
    HIP_TRY(hipEventRecord(o.ready, o.cap));
    HIP_TRY(hipStreamWaitEvent(st, o.ready, 0));
    HIP_TRY(hipStreamSynchronize(o.cap));
    return GPMPPI_OK;
}

// Phi^-1(p): the upper-tail probability q = min(p, 1-p) is inverted by
// bisection on 0.5 erfc(z / sqrt 2) = q over [0, 40], refined by Newton steps.
double norm_quantile(double p) {
    const double q = p < 0.5 ? p : 1.0 - p;
    auto tail = [](double z) { return 0.5 * std::erfc(z / std::sqrt(2.0)); };
    double lo = 0.0, hi = 40.0;
    for (int i = 0; i < 200; ++i) {
        const double mid = 0.5 * (lo + hi);
        if (tail(mid) > q) lo = mid; else hi = mid;
    }
    double z = 0.5 * (lo + hi);
    for (int i = 0; i < 3; ++i) {
        const double phi = std::exp(-0.5 * z * z) / std::sqrt(2.0 * M_PI);
        if (phi > 0) z += (tail(z) - q) / phi;
    }
    return p < 0.5 ? -z : z;
}

template <typename T>
T *dev_alloc(size_t n, gpmppi_status &st) {
    void *p = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
        st = fail(GPMPPI_E_NOMEM, "hipMalloc of %zu bytes failed", n * sizeof(T));
        return nullptr;
    }
    return static_cast<T *>(p);
}

}  // namespace

namespace gpmppi {
gpmppi_status set_error(gpmppi_status st, const char *msg) { return fail(st, "%s", msg); }
}  // namespace gpmppi

constexpr int kGradMaxMpad = 512;   // the adjoint's LDS plan holds k and r for 32 samples

// Scratch memory of the allocation-free entry point (gpmppi_grad_noalloc): one
// array per GPU the library runs on, held until the process ends and shared by
// every call on that GPU.  Host code never uses this name as an address: each
// device's address comes from scratch_address() and is kept per device.
constexpr size_t kScratchBytes = size_t(GPMPPI_GRAD_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up once per
// device (with that device current) and kept.
gpmppi_status scratch_address(int dev, void **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return fail(GPMPPI_E_UNSUPPORTED, "device %d is beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(GPMPPI_E_HIP, "hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GPMPPI_OK;
}

}  // namespace

struct gpmppi_ctx {
    int device = 0;
    gpmppi_params params{};
    int M = 0, Mpad = 0, NT = 0;
    double z_p = 0, c_p = 0;
    // device buffers
    float *zs = nullptr, *alpha = nullptr, *zs2 = nullptr, *cz = nullptr;
    int groups = 1;                  // sample groups of 32 per rollout workgroup (tuned)
    int waves = 4;                   // wave64s per rollout workgroup, 4 or 8 (tuned)
    int rotate = 1;                  // block-dependent start of the walk over W (tuned)
    int split = 0;                   // 1: the two GP outputs of a sample block on two workgroups (tuned)
    unsigned long long *xrec = nullptr;   // output-split exchange records [ceil(K/32)][kXchRecPerBlock]
    uint32_t *xep = nullptr;              // output-split launch epoch and finished-workgroup count
    uint32_t *repair = nullptr;           // output-split blocks left to the repair launch [ceil(K/32)], zero between launches
    int xspin = kXchSpin;                 // polls per output-split exchange wait
    float4 *w32 = nullptr;
    uint4 *wbh = nullptr, *wbl = nullptr;
    uint4 *zop = nullptr;            // BF16 exponent-product operands per output
    long long w32_stride = 0, wb_stride = 0, zop_stride = 0;
    float4 *q32 = nullptr;           // dense packed Q = A^-1 per output (differentiation form, Mpad <= 512)
    long long q_stride = 0;          // float4 per output
    void *grad_ws = nullptr;         // differentiation-form workspace (grown on demand)
    int grad_split = 1;              // 1: split the gradient's outputs over two workgroups where they fit
    size_t grad_ws_bytes = 0;
    void *scratch = nullptr;         // this device's allocation-free scratch array (not owned)
    float4 *obs = nullptr;
    float4 *seg = nullptr;
    float *seg_inv = nullptr;
    uint32_t *flags = nullptr;       // [0] status bits, [1] non-PD flag, [2] closed-loop step counter
    double *A64 = nullptr, *W64 = nullptr, *Z64 = nullptr, *y64 = nullptr, *u64 = nullptr, *al64 = nullptr;
    // terrain ensemble (Eq. 3): per-terrain alpha on shared inputs and hyperparameters
    int n_terr = 0;
    double *alpha_terr = nullptr;    // [2][n_terr][Mpad] FP64 (output-major)
    std::vector<double> Zh[2], yh[2];
    double log_ell[2][4] = {}, log_sf[2] = {}, log_sn[2] = {};
    float *U_scratch = nullptr;      // [T][2] new controls inside the closed loop
    float *cost_scratch = nullptr;   // [K]
    float *tight = nullptr;          // [T+1][3] nominal Sigma_XY (Step 2 tightening)
    // host copies
    GpDev gp{};
    Geometry geo{};
    CostWeights cw{};
    Dyn dyn{};
    int n_obs = 0;
    std::vector<void *> owned;

    ~gpmppi_ctx() {
        if (grad_ws) (void)hipFree(grad_ws);
        for (void *p : owned) (void)hipFree(p);
    }
};

namespace {

gpmppi_status validate_params(const gpmppi_params *p) {
    if (!p) return fail(GPMPPI_E_INVALID, "params is NULL");
    if (p->K < 1) return fail(GPMPPI_E_INVALID, "K must be >= 1 (got %d)", p->K);
    if (p->K > (1 << 24)) return fail(GPMPPI_E_UNSUPPORTED, "K must be <= 2^24 (got %d)", p->K);
    if (p->T < 1 || p->T > 4096) return fail(GPMPPI_E_INVALID, "T must lie in [1, 4096] (got %d)", p->T);
    const double vals[] = {p->dt, p->tau_v, p->tau_w, p->sig_v, p->sig_w, p->u_min[0], p->u_min[1],
                           p->u_max[0], p->u_max[1], p->lambda, p->p_x, p->w_var, p->w_dev, p->w_lane,
                           p->w_speed, p->w_obs, p->v_des, p->discount};
    for (double v : vals)
        if (!is_fin(v)) return fail(GPMPPI_E_NONFINITE, "non-finite controller parameter");
    if (!(p->dt > 0) || !(p->tau_v > 0) || !(p->tau_w > 0))
        return fail(GPMPPI_E_INVALID, "dt, tau_v and tau_w must be > 0");
    if (p->sig_v < 0 || p->sig_w < 0) return fail(GPMPPI_E_INVALID, "noise scales must be >= 0");
    if (!(p->u_min[0] < p->u_max[0]) || !(p->u_min[1] < p->u_max[1]))
        return fail(GPMPPI_E_INVALID, "u_min must be < u_max");
    if (!(p->lambda > 0)) return fail(GPMPPI_E_INVALID, "lambda must be > 0");
    if (!(p->p_x > 0 && p->p_x < 1)) return fail(GPMPPI_E_INVALID, "p_x must lie in (0, 1)");
    if (p->precision < 0 || p->precision > 2) return fail(GPMPPI_E_INVALID, "unknown precision %d", p->precision);
    if (p->problem_id < 0) return fail(GPMPPI_E_INVALID, "problem_id must be >= 0");
    if (!is_fin(p->w_goal) || !is_fin(p->w_term) || !is_fin(p->goal[0]) || !is_fin(p->goal[1]) ||
        !is_fin(p->goal_tol))
        return fail(GPMPPI_E_NONFINITE, "non-finite goal parameter");
    if (p->w_goal < 0 || p->w_term < 0 || !(p->goal_tol > 0))
        return fail(GPMPPI_E_INVALID, "goal weights must be >= 0 and goal_tol > 0");
    if (p->tighten != 0 && p->tighten != 1) return fail(GPMPPI_E_INVALID, "tighten must be 0 or 1");
    return GPMPPI_OK;
}

gpmppi_status validate_gp(const gpmppi_gp gp[2]) {
    if (!gp) return fail(GPMPPI_E_INVALID, "gp is NULL");
    if (gp[0].M != gp[1].M) return fail(GPMPPI_E_INVALID, "both GPs must have the same M");
    for (int o = 0; o < 2; ++o) {
        const gpmppi_gp &g = gp[o];
        if (g.M < 1) return fail(GPMPPI_E_INVALID, "GP %d: M must be >= 1", o);
        if (g.M > kMaxM) return fail(GPMPPI_E_UNSUPPORTED, "GP %d: M = %d exceeds %d", o, g.M, kMaxM);
        if (!g.Z || !g.y) return fail(GPMPPI_E_INVALID, "GP %d: Z or y is NULL", o);
        for (int i = 0; i < 4 * g.M; ++i)
            if (!is_fin(g.Z[i])) return fail(GPMPPI_E_NONFINITE, "GP %d: non-finite input Z", o);
        for (int i = 0; i < g.M; ++i)
            if (!is_fin(g.y[i])) return fail(GPMPPI_E_NONFINITE, "GP %d: non-finite target y", o);
        for (int d = 0; d < 4; ++d)
            if (!is_fin(g.log_ell[d]) || std::fabs(g.log_ell[d]) > 30)
                return fail(GPMPPI_E_INVALID, "GP %d: log lengthscale out of range", o);
        if (!is_fin(g.log_sf) || std::fabs(g.log_sf) > 30 || !is_fin(g.log_sn) || std::fabs(g.log_sn) > 30)
            return fail(GPMPPI_E_INVALID, "GP %d: log sigma out of range", o);
    }
    return GPMPPI_OK;
}

gpmppi_status validate_world(const gpmppi_obstacles *ob, const gpmppi_path *pa) {
    if (!ob || !pa) return fail(GPMPPI_E_INVALID, "obstacles or path is NULL");
    if (ob->n < 0 || ob->n > 4096) return fail(GPMPPI_E_INVALID, "obstacle count must lie in [0, 4096]");
    if (ob->n > 0 && !ob->xyr) return fail(GPMPPI_E_INVALID, "obstacle array is NULL");
    for (int j = 0; j < ob->n; ++j) {
        for (int c = 0; c < 3; ++c)
            if (!is_fin(ob->xyr[3 * j + c])) return fail(GPMPPI_E_NONFINITE, "non-finite obstacle");
        if (!(ob->xyr[3 * j + 2] > 0)) return fail(GPMPPI_E_INVALID, "obstacle radius must be > 0");
    }
    if (!is_fin(pa->half_width) || !(pa->half_width > 0))
        return fail(GPMPPI_E_INVALID, "lane half-width must be > 0");
    if (pa->kind == 0) {
        if (!is_fin(pa->cx) || !is_fin(pa->cy) || !is_fin(pa->R) || !(pa->R > 0))
            return fail(GPMPPI_E_INVALID, "circle path needs finite centre and R > 0");
    } else if (pa->kind == 1) {
        if (pa->P < 3 || pa->P > 65536 || !pa->pts) return fail(GPMPPI_E_INVALID, "polyline needs 3..65536 vertices");
        for (int i = 0; i < 2 * pa->P; ++i)
            if (!is_fin(pa->pts[i])) return fail(GPMPPI_E_NONFINITE, "non-finite path vertex");
        for (int i = 0; i < pa->P; ++i) {
            const int n = (i + 1) % pa->P;
            if (pa->pts[2 * i] == pa->pts[2 * n] && pa->pts[2 * i + 1] == pa->pts[2 * n + 1])
                return fail(GPMPPI_E_INVALID, "polyline has a zero-length segment at vertex %d", i);
        }
    } else {
        return fail(GPMPPI_E_INVALID, "unknown path kind %d", pa->kind);
    }
    return GPMPPI_OK;
}

gpmppi_status build_gps(gpmppi_ctx *c, const gpmppi_gp gp[2]) {
    const int M = c->M, Mpad = c->Mpad;
    for (int o = 0; o < 2; ++o) {
        c->Zh[o].assign(gp[o].Z, gp[o].Z + 4 * M);
        c->yh[o].assign(gp[o].y, gp[o].y + M);
        for (int d = 0; d < 4; ++d) c->log_ell[o][d] = gp[o].log_ell[d];
        c->log_sf[o] = gp[o].log_sf;
        c->log_sn[o] = gp[o].log_sn;
    }
    c->n_terr = 0;
    const double kScale = std::sqrt(0.5 / std::log(2.0));   // sqrt(log2(e) / 2)
    for (int o = 0; o < 2; ++o) {
        std::vector<double> y(Mpad, 0.0);
        std::memcpy(y.data(), gp[o].y, sizeof(double) * M);
        HIP_TRY(hipMemcpy(c->Z64, gp[o].Z, sizeof(double) * 4 * M, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->y64, y.data(), sizeof(double) * Mpad, hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(c->flags + 1, 0, sizeof(uint32_t)));
        double ell[4], scale[4];
        for (int d = 0; d < 4; ++d) {
            ell[d] = std::exp(gp[o].log_ell[d]);
            scale[d] = kScale / ell[d];
        }
        const double sf2 = std::exp(2.0 * gp[o].log_sf), sn2 = std::exp(2.0 * gp[o].log_sn);
        GpBuildBuffers b{c->A64, c->W64, c->Z64, c->y64, c->u64, c->al64, c->flags + 1};
        HIP_TRY(build_gp_output(b, M, Mpad, ell, sf2, sn2, nullptr));
        uint32_t notpd = 0;
        HIP_TRY(hipMemcpy(&notpd, c->flags + 1, sizeof notpd, hipMemcpyDeviceToHost));
        if (notpd) return fail(GPMPPI_E_NOT_PD, "GP %d: K(Z,Z) + sn^2 I is not positive definite", o);
        const double c2 = 2.0 * gp[o].log_sf / std::log(2.0);
        HIP_TRY(pack_gp_output(b, M, Mpad, scale, c2, c->zop + o * c->zop_stride, c->zs + (size_t)o * Mpad * 4,
                               c->alpha + (size_t)o * Mpad,
                               c->zs2 + (size_t)o * Mpad * 4, c->cz + (size_t)o * Mpad,
                               c->w32 + o * c->w32_stride, c->wbh + o * c->wb_stride, c->wbl + o * c->wb_stride,
                               nullptr));
        if (c->q32) HIP_TRY(pack_q(b, M, Mpad, c->q32 + (size_t)o * c->q_stride, nullptr));
        HIP_TRY(hipDeviceSynchronize());
        for (int d = 0; d < 4; ++d) c->gp.scale[o][d] = (float)scale[d];
        c->gp.c2[o] = (float)(2.0 * gp[o].log_sf / std::log(2.0));
        c->gp.sf2[o] = (float)sf2;
        c->gp.sn2[o] = (float)sn2;
        c->gp.vscale[o] = 1.0f;
    }
    return GPMPPI_OK;
}

NoiseParams noise_of(const gpmppi_ctx *c) {
    NoiseParams np{};
    np.pid = (uint32_t)c->params.problem_id;
    np.sig_v = (float)c->params.sig_v;
    np.sig_w = (float)c->params.sig_w;
    np.umin0 = (float)c->params.u_min[0];
    np.umin1 = (float)c->params.u_min[1];
    np.umax0 = (float)c->params.u_max[0];
    np.umax1 = (float)c->params.u_max[1];
    return np;
}

RolloutArgs rollout_args(const gpmppi_ctx *c, const float *x0, const float *U, uint64_t seed, float *costs,
                         const gpmppi_trace *trace, const uint32_t *step_counter) {
    RolloutArgs a{};
    a.gp = c->gp;
    a.geo = c->geo;
    a.cw = c->cw;
    a.dyn = c->dyn;
    a.noise = noise_of(c);
    a.seed = seed;
    a.step_counter = step_counter;
    a.K = c->params.K;
    a.T = c->params.T;
    a.rotate = c->rotate;
    a.xrec = c->xrec;
    a.xep = c->xep;
    a.xspin = c->xspin;
    a.flags = c->flags;
    a.repair = c->repair;
    a.x0 = x0;
    a.U = U;
    a.costs = costs;
    if (trace) a.trace = *trace;
    return a;
}

// Alg. 1 Step 2: one zero-noise sample along clip(U) writes Sigma_XY per step
// into c->tight; returns the table pointer for the main rollout (or NULL).
const float *enqueue_tightening(gpmppi_ctx *c, const float *x0, const float *U, const uint32_t *step_counter,
                                hipStream_t st, hipError_t &err) {
    err = hipSuccess;
    if (c->params.tighten != 1) return nullptr;
    RolloutArgs n = rollout_args(c, x0, U, 0, c->cost_scratch, nullptr, step_counter);
    n.K = 1;
    n.noise.sig_v = 0.0f;
    n.noise.sig_w = 0.0f;
    n.trace.sxy_d = c->tight;
    err = launch_rollout(n, c->params.precision, c->groups, c->waves, c->split, st);
    return c->tight;
}

UpdateArgs update_args(const gpmppi_ctx *c, const float *costs, const float *U, uint64_t seed, float *U_out,
                       float *weights, const uint32_t *step_counter) {
    UpdateArgs u{};
    u.noise = noise_of(c);
    u.seed = seed;
    u.step_counter = step_counter;
    u.K = c->params.K;
    u.T = c->params.T;
    u.lambda = (float)c->params.lambda;
    u.costs = costs;
    u.U = U;
    u.U_out = U_out;
    u.weights = weights;
    u.flags = c->flags;
    return u;
}

}  // namespace

extern "C" {

const char *gpmppi_last_error(void) { return g_last_error.c_str(); }

gpmppi_status gpmppi_init(const gpmppi_params *params, const gpmppi_gp gp[2], const gpmppi_obstacles *obstacles,
                          const gpmppi_path *path, gpmppi_ctx **out) {
    g_last_error.clear();
    if (!out) return fail(GPMPPI_E_INVALID, "out is NULL");
    gpmppi_status st;
    if ((st = validate_params(params)) != GPMPPI_OK) return st;
    if ((st = validate_gp(gp)) != GPMPPI_OK) return st;
    if ((st = validate_world(obstacles, path)) != GPMPPI_OK) return st;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(GPMPPI_E_HIP, "no HIP device available");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    void *scratch_ptr = nullptr;
    if ((st = scratch_address(dev, &scratch_ptr)) != GPMPPI_OK) return st;
    auto *c = new gpmppi_ctx();
    c->device = dev;
    c->scratch = scratch_ptr;
    c->params = *params;
    c->M = gp[0].M;
    c->Mpad = (c->M + 63) / 64 * 64;   // an even number of 32-row tiles (pairs of row tiles)
    c->NT = c->Mpad / 32;
    const int Mpad = c->Mpad, NT = c->NT;
    const int NP = (NT + 1) / 2;   // row-tile pairs; pair u holds 2 (2u + 2) blocks
    c->w32_stride = (long long)2 * NP * (NP + 1) * 256;
    c->wb_stride = (long long)2 * NP * (NP + 1) * 128;
    c->n_obs = obstacles->n;
    const int P = path->kind == 1 ? path->P : 0;

    st = GPMPPI_OK;
    auto track = [&](auto *p) {
        if (p) c->owned.push_back((void *)p);
        return p;
    };
    c->zs = track(dev_alloc<float>((size_t)2 * Mpad * 4, st));
    c->alpha = track(dev_alloc<float>((size_t)2 * Mpad, st));
    c->zs2 = track(dev_alloc<float>((size_t)2 * Mpad * 4, st));
    c->cz = track(dev_alloc<float>((size_t)2 * Mpad, st));
    c->w32 = track(dev_alloc<float4>((size_t)2 * c->w32_stride, st));
    c->wbh = track(dev_alloc<uint4>((size_t)2 * c->wb_stride, st));
    c->wbl = track(dev_alloc<uint4>((size_t)2 * c->wb_stride, st));
    c->zop_stride = (long long)(Mpad / 32) * 128;
    c->zop = track(dev_alloc<uint4>((size_t)2 * c->zop_stride, st));
    if (Mpad <= kGradMaxMpad) {
        c->q_stride = (long long)(Mpad / 32) * (Mpad / 32) * 256;
        c->q32 = track(dev_alloc<float4>((size_t)2 * c->q_stride, st));
    }
    c->obs = track(dev_alloc<float4>((size_t)std::max(1, c->n_obs), st));
    c->seg = track(dev_alloc<float4>((size_t)std::max(1, P), st));
    c->seg_inv = track(dev_alloc<float>((size_t)std::max(1, P), st));
    c->flags = track(dev_alloc<uint32_t>(4, st));
    c->A64 = track(dev_alloc<double>((size_t)Mpad * Mpad, st));
    c->W64 = track(dev_alloc<double>((size_t)Mpad * Mpad, st));
    c->Z64 = track(dev_alloc<double>((size_t)Mpad * 4, st));
    c->y64 = track(dev_alloc<double>((size_t)Mpad, st));
    c->u64 = track(dev_alloc<double>((size_t)Mpad, st));
    c->al64 = track(dev_alloc<double>((size_t)Mpad, st));
    c->U_scratch = track(dev_alloc<float>((size_t)2 * params->T, st));
    c->cost_scratch = track(dev_alloc<float>((size_t)params->K, st));
    c->tight = track(dev_alloc<float>((size_t)3 * (params->T + 1) + 1, st));
    const size_t nxrec = (size_t)((params->K + 31) / 32) * kXchRecPerBlock;
    c->xrec = track(dev_alloc<unsigned long long>(nxrec, st));
    c->xep = track(dev_alloc<uint32_t>(2, st));
    const size_t nblk = (size_t)((params->K + 31) / 32);
    c->repair = track(dev_alloc<uint32_t>(nblk, st));
    if (st != GPMPPI_OK) {
        delete c;
        return st;
    }
    if (hipMemset(c->flags, 0, 4 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->xrec, 0, nxrec * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->xep, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->repair, 0, nblk * sizeof(uint32_t)) != hipSuccess) {
        delete c;
        return fail(GPMPPI_E_HIP, "hipMemset failed");
    }

    // world geometry in FP32
    std::vector<float4> obs(std::max(1, c->n_obs));
    for (int j = 0; j < c->n_obs; ++j)
        obs[j] = make_float4((float)obstacles->xyr[3 * j], (float)obstacles->xyr[3 * j + 1],
                             (float)obstacles->xyr[3 * j + 2], 0.0f);
    std::vector<float4> seg(std::max(1, P));
    std::vector<float> seg_inv(std::max(1, P), 0.0f);
    for (int i = 0; i < P; ++i) {
        const int n = (i + 1) % P;
        const double ax = path->pts[2 * i], ay = path->pts[2 * i + 1];
        const double ex = path->pts[2 * n] - ax, ey = path->pts[2 * n + 1] - ay;
        seg[i] = make_float4((float)ax, (float)ay, (float)ex, (float)ey);
        seg_inv[i] = (float)(1.0 / (ex * ex + ey * ey));
    }
    if (hipMemcpy(c->obs, obs.data(), sizeof(float4) * obs.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->seg, seg.data(), sizeof(float4) * seg.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->seg_inv, seg_inv.data(), sizeof(float) * seg_inv.size(), hipMemcpyHostToDevice) != hipSuccess) {
        delete c;
        return fail(GPMPPI_E_HIP, "upload of the world geometry failed");
    }
    c->z_p = norm_quantile(params->p_x);
    c->c_p = std::sqrt(-2.0 * std::log1p(-params->p_x));

    c->gp.zs = c->zs;
    c->gp.alpha = c->alpha;
    c->gp.w32 = c->w32;
    c->gp.wbh = c->wbh;
    c->gp.wbl = c->wbl;
    c->gp.w32_stride = c->w32_stride;
    c->gp.wb_stride = c->wb_stride;
    c->gp.zop = c->zop;
    c->gp.zop_stride = c->zop_stride;
    c->gp.Mpad = Mpad;
    c->groups = rollout_groups(params->precision, Mpad);
    c->gp.NT = NT;

    Geometry &g = c->geo;
    g.path_kind = path->kind;
    g.cx = (float)path->cx;
    g.cy = (float)path->cy;
    g.R = (float)path->R;
    g.P = P;
    g.seg = c->seg;
    g.seg_inv = c->seg_inv;
    g.half_width = (float)path->half_width;
    g.inv_half_width = (float)(1.0 / path->half_width);
    g.n_obs = c->n_obs;
    g.obs = c->obs;
    g.z_p = (float)c->z_p;
    g.c_p = (float)c->c_p;

    c->cw = CostWeights{(float)params->w_var, (float)params->w_dev, (float)params->w_lane, (float)params->w_speed,
                        (float)params->w_obs, (float)params->v_des, (float)params->discount,
                        (float)params->w_goal, (float)params->w_term, (float)params->goal[0],
                        (float)params->goal[1], (float)params->goal_tol};
    c->dyn = Dyn{(float)params->dt, (float)(params->dt / params->tau_v), (float)(params->dt / params->tau_w),
                 (float)(1.0 - params->dt / params->tau_v), (float)(1.0 - params->dt / params->tau_w)};

    if ((st = build_gps(c, gp)) != GPMPPI_OK) {
        delete c;
        return st;
    }
    *out = c;
    return GPMPPI_OK;
}

gpmppi_status gpmppi_set_gp(gpmppi_ctx *c, const gpmppi_gp gp[2]) {
    g_last_error.clear();
    if (!c) return fail(GPMPPI_E_INVALID, "ctx is NULL");
    gpmppi_status st;
    if ((st = validate_gp(gp)) != GPMPPI_OK) return st;
    if (gp[0].M != c->M) return fail(GPMPPI_E_INVALID, "M must stay %d (got %d)", c->M, gp[0].M);
    return build_gps(c, gp);
}

gpmppi_status gpmppi_set_terrains(gpmppi_ctx *c, int32_t n_terr, const double *y, const double *w) {
    g_last_error.clear();
    if (!c || !y || !w) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n_terr < 1 || n_terr > 8) return fail(GPMPPI_E_INVALID, "terrain count must lie in [1, 8]");
    const int M = c->M, Mpad = c->Mpad;
    for (long long i = 0; i < (long long)n_terr * 2 * M; ++i)
        if (!is_fin(y[i])) return fail(GPMPPI_E_NONFINITE, "non-finite terrain target");
    for (int i = 0; i < n_terr; ++i)
        if (!is_fin(w[i])) return fail(GPMPPI_E_NONFINITE, "non-finite terrain weight");
    if (c->alpha_terr) {
        (void)hipFree(c->alpha_terr);
        c->owned.erase(std::remove(c->owned.begin(), c->owned.end(), (void *)c->alpha_terr), c->owned.end());
        c->alpha_terr = nullptr;
    }
    gpmppi_status st = GPMPPI_OK;
    // layout [o][i][Mpad] so that one output's terrains are contiguous
    c->alpha_terr = dev_alloc<double>((size_t)2 * n_terr * Mpad, st);
    if (st != GPMPPI_OK) return st;
    c->owned.push_back(c->alpha_terr);
    std::vector<double> yp(Mpad, 0.0);
    for (int o = 0; o < 2; ++o) {
        // factor this output once (the targets do not enter L or W), then one alpha per terrain
        double ell[4];
        for (int d = 0; d < 4; ++d) ell[d] = std::exp(c->log_ell[o][d]);
        HIP_TRY(hipMemcpy(c->Z64, c->Zh[o].data(), sizeof(double) * 4 * M, hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(c->y64, 0, sizeof(double) * Mpad));
        HIP_TRY(hipMemset(c->flags + 1, 0, sizeof(uint32_t)));
        GpBuildBuffers b{c->A64, c->W64, c->Z64, c->y64, c->u64, c->al64, c->flags + 1};
        HIP_TRY(build_gp_output(b, M, Mpad, ell, std::exp(2.0 * c->log_sf[o]), std::exp(2.0 * c->log_sn[o]),
                                nullptr));
        uint32_t notpd = 0;
        HIP_TRY(hipMemcpy(&notpd, c->flags + 1, sizeof notpd, hipMemcpyDeviceToHost));
        if (notpd) return fail(GPMPPI_E_NOT_PD, "GP %d: K(Z,Z) + sn^2 I is not positive definite", o);
        for (int i = 0; i < n_terr; ++i) {
            std::fill(yp.begin(), yp.end(), 0.0);
            std::memcpy(yp.data(), y + ((size_t)i * 2 + o) * M, sizeof(double) * M);
            HIP_TRY(hipMemcpy(c->y64, yp.data(), sizeof(double) * Mpad, hipMemcpyHostToDevice));
            HIP_TRY(alpha_for_targets(b, Mpad, c->y64, c->alpha_terr + ((size_t)o * n_terr + i) * Mpad, nullptr));
            HIP_TRY(hipDeviceSynchronize());
        }
    }
    c->n_terr = n_terr;
    return gpmppi_set_terrain_weights(c, w);
}

gpmppi_status gpmppi_set_terrain_weights(gpmppi_ctx *c, const double *w) {
    g_last_error.clear();
    if (!c || !w) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (c->n_terr < 1) return fail(GPMPPI_E_INVALID, "no terrains set (gpmppi_set_terrains)");
    for (int i = 0; i < c->n_terr; ++i)
        if (!is_fin(w[i])) return fail(GPMPPI_E_NONFINITE, "non-finite terrain weight");
    TerrainWeights tw{};
    double s2 = 0.0;
    for (int i = 0; i < c->n_terr; ++i) {
        tw.w[i] = w[i];
        s2 += w[i] * w[i];
    }
    const int Mpad = c->Mpad;
    for (int o = 0; o < 2; ++o) {
        HIP_TRY(combine_alpha(c->alpha_terr + (size_t)o * c->n_terr * Mpad, c->n_terr, Mpad, tw, nullptr,
                              c->alpha + (size_t)o * Mpad, nullptr));
        c->gp.vscale[o] = (float)s2;
    }
    HIP_TRY(hipDeviceSynchronize());
    return GPMPPI_OK;
}

gpmppi_status gpmppi_terrain_means(gpmppi_ctx *c, const float *q_d, int32_t n, float *out_d, void *stream) {
    g_last_error.clear();
    if (!c || !q_d || !out_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n < 1) return fail(GPMPPI_E_INVALID, "n must be >= 1");
    if (c->n_terr < 1) return fail(GPMPPI_E_INVALID, "no terrains set (gpmppi_set_terrains)");
    HIP_TRY(launch_terrain_means(q_d, n, c->gp, c->alpha_terr, c->n_terr, out_d, (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_rollout(gpmppi_ctx *c, const float *x0_d, const float *U_d, uint64_t seed, float *costs_d,
                             const gpmppi_trace *trace, void *stream) {
    g_last_error.clear();
    if (!c || !x0_d || !U_d || !costs_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    hipError_t e;
    const float *tight = enqueue_tightening(c, x0_d, U_d, nullptr, (hipStream_t)stream, e);
    HIP_TRY(e);
    RolloutArgs a = rollout_args(c, x0_d, U_d, seed, costs_d, trace, nullptr);
    a.tight_sxy = tight;
    HIP_TRY(launch_rollout(a, c->params.precision, c->groups, c->waves, c->split, (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_weights_update(gpmppi_ctx *c, const float *costs_d, const float *U_d, uint64_t seed,
                                    float *U_out_d, float *weights_d, void *stream) {
    g_last_error.clear();
    if (!c || !costs_d || !U_d || !U_out_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    const UpdateArgs u = update_args(c, costs_d, U_d, seed, U_out_d, weights_d, nullptr);
    HIP_TRY(launch_update(u, (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_step(gpmppi_ctx *c, const float *x0_d, const float *U_d, uint64_t seed, float *U_out_d,
                          float *costs_d, float *weights_d, void *stream) {
    g_last_error.clear();
    if (!c || !x0_d || !U_d || !U_out_d || !costs_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    hipError_t e;
    const float *tight = enqueue_tightening(c, x0_d, U_d, nullptr, (hipStream_t)stream, e);
    HIP_TRY(e);
    RolloutArgs a = rollout_args(c, x0_d, U_d, seed, costs_d, nullptr, nullptr);
    a.tight_sxy = tight;
    HIP_TRY(launch_rollout(a, c->params.precision, c->groups, c->waves, c->split, (hipStream_t)stream));
    const UpdateArgs u = update_args(c, costs_d, U_d, seed, U_out_d, weights_d, nullptr);
    HIP_TRY(launch_update(u, (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_gp_predict(gpmppi_ctx *c, const float *q_d, int32_t n, float *mean_d, float *var_d,
                                void *stream) {
    g_last_error.clear();
    if (!c || !q_d || !mean_d || !var_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n < 1) return fail(GPMPPI_E_INVALID, "n must be >= 1");
    HIP_TRY(launch_gp_predict(c->gp, c->params.precision, q_d, n, mean_d, var_d, (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_plant_shift(gpmppi_ctx *c, const float *x_d, float *x_out_d, float *U_d, double amplitude,
                                 void *stream) {
    g_last_error.clear();
    if (!c || !x_d || !x_out_d || !U_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (!is_fin(amplitude)) return fail(GPMPPI_E_NONFINITE, "non-finite plant amplitude");
    HIP_TRY(launch_plant_shift(x_d, x_out_d, U_d, c->params.T, c->dyn, (float)amplitude, nullptr, nullptr, nullptr,
                               (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_closed_loop(gpmppi_ctx *c, float *x_d, float *U_d, uint64_t seed0, int32_t n,
                                 double amplitude, float *x_hist_d, float *U0_hist_d, int32_t use_graph,
                                 void *stream) {
    g_last_error.clear();
    if (!c || !x_d || !U_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n < 0) return fail(GPMPPI_E_INVALID, "n must be >= 0");
    if (!is_fin(amplitude)) return fail(GPMPPI_E_NONFINITE, "non-finite plant amplitude");
    hipStream_t st = (hipStream_t)stream;
    uint32_t *counter = c->flags + 2;
    HIP_TRY(launch_counter_reset(counter, st));
    if (x_hist_d) HIP_TRY(hipMemcpyAsync(x_hist_d, x_d, 5 * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (n == 0) return GPMPPI_OK;
    // one control step: rollout -> weights/update -> plant + shift, keyed by seed0 + counter
    auto enqueue = [&](hipStream_t s) -> gpmppi_status {
        hipError_t e;
        const float *tight = enqueue_tightening(c, x_d, U_d, counter, s, e);
        HIP_TRY(e);
        RolloutArgs a = rollout_args(c, x_d, U_d, seed0, c->cost_scratch, nullptr, counter);
        a.tight_sxy = tight;
        HIP_TRY(launch_rollout(a, c->params.precision, c->groups, c->waves, c->split, s));
        const UpdateArgs u = update_args(c, c->cost_scratch, U_d, seed0, U_d, nullptr, counter);
        HIP_TRY(launch_update(u, s));
        HIP_TRY(launch_plant_shift(x_d, x_d, U_d, c->params.T, c->dyn, (float)amplitude, counter, x_hist_d,
                                   U0_hist_d, s));
        return GPMPPI_OK;
    };
    if (!use_graph) {
        for (int t = 0; t < n; ++t) {
            gpmppi_status s = enqueue(st);
            if (s != GPMPPI_OK) return s;
        }
        return GPMPPI_OK;
    }
    return replay_captured(st, n, enqueue);
}

gpmppi_status gpmppi_philox(uint64_t seed, const uint32_t *ctr_d, int32_t n, uint32_t *out_d, void *stream) {
    g_last_error.clear();
    if (!ctr_d || !out_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n < 1) return fail(GPMPPI_E_INVALID, "n must be >= 1");
    HIP_TRY(launch_philox(seed, ctr_d, n, out_d, (hipStream_t)stream));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_status_flags(gpmppi_ctx *c, uint32_t *flags) {
    g_last_error.clear();
    if (!c || !flags) return fail(GPMPPI_E_INVALID, "NULL argument");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(flags, c->flags, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(c->flags, 0, sizeof(uint32_t)));
    return GPMPPI_OK;
}

gpmppi_status gpmppi_info(const gpmppi_ctx *c, int32_t *M_pad, double *z_p, double *c_p) {
    g_last_error.clear();
    if (!c) return fail(GPMPPI_E_INVALID, "ctx is NULL");
    if (M_pad) *M_pad = c->Mpad;
    if (z_p) *z_p = c->z_p;
    if (c_p) *c_p = c->c_p;
    return GPMPPI_OK;
}

// ------------------------------------------------------------------ batch
}  // extern "C"

struct gpmppi_batch {
    int n = 0, precision = 0, Mpad_max = 0, grid = 0, cus = 1;
    int G = 1, G_max = 1, rotate = 1, wg_per_cu = 1, wg_per_cu_max = 1, order = 0, waves = 4;
    std::vector<gpmppi_ctx *> ctx;
    std::vector<long long> U_off, K_off;   // n + 1 each
    std::vector<double> cost;              // estimated rollout cost of one sample block, per problem
    std::vector<RolloutArgs> ra_h;         // host copy of the per-problem rollout arguments
    int n_items = 0, n_upd = 0;
    RolloutArgs *ra = nullptr;      // [n] device
    UpdateArgs *ua = nullptr;       // [n] device
    int2 *items = nullptr;          // rollout items (problem, block); sized for one group per block
    int2 *upd_items = nullptr;      // update items (problem, step)
    long long *U_off_d = nullptr, *K_off_d = nullptr;
    int *T_d = nullptr;
    Dyn *dyn_d = nullptr;
    uint32_t *counters = nullptr;   // [0] work counter, [1] closed-loop step
    float *cost_scratch = nullptr;
    float *U_scratch = nullptr;     // packed controls written by the tuner's updates (never read)
    std::vector<void *> owned;
    ~gpmppi_batch() {
        for (void *p : owned) (void)hipFree(p);
        for (gpmppi_ctx *c : ctx) delete c;
    }
};

namespace {

gpmppi_status batch_enqueue_step(gpmppi_batch *b, hipStream_t st) {
    HIP_TRY(launch_counter_reset(b->counters, st));
    HIP_TRY(launch_rollout_batch(b->ra, b->items, b->n_items, b->counters, b->precision, b->G, b->waves,
                                 b->Mpad_max, b->grid, st));
    HIP_TRY(launch_update_batch(b->ua, b->upd_items, b->n_upd, st));
    return GPMPPI_OK;
}

// Most persistent workgroups one compute unit holds at this LDS plan (at most 2).
int wg_capacity(int precision, int G, int Mpad) {
    const size_t lds = rollout_lds_bytes(precision, G, Mpad);
    return std::max(1, std::min(2, (int)((160 * 1024) / (lds + 4096))));
}

// Both workgroups of every sample block fit the device at once (output split, one group).
bool split_admissible(const gpmppi_ctx *c, int waves) {
    return c->params.K <= rollout_split_capacity(c->params.precision, c->Mpad, waves);
}

gpmppi_status check_tuning(const gpmppi_tuning *t, int G_max, int wg_max, bool batch) {
    if (!t) return fail(GPMPPI_E_INVALID, "tuning is NULL");
    if (t->waves != 4 && t->waves != 8 && t->waves != kPipeWaves)
        return fail(GPMPPI_E_INVALID, "waves must be 4, 8 or %d (got %d)", kPipeWaves, t->waves);
    if (t->waves == kPipeWaves && batch) return fail(GPMPPI_E_INVALID, "batches run 4 or 8 waves per workgroup");
    if (t->waves == kPipeWaves && t->split) return fail(GPMPPI_E_INVALID, "the wave-specialised rollout does not split outputs");
    if (t->groups < 1 || t->groups > G_max)
        return fail(GPMPPI_E_INVALID, "groups must lie in [1, %d] here (got %d)", G_max, t->groups);
    if (t->rotate != 0 && t->rotate != 1) return fail(GPMPPI_E_INVALID, "rotate must be 0 or 1");
    if (t->split != 0 && t->split != 1) return fail(GPMPPI_E_INVALID, "split must be 0 or 1");
    if (t->split && batch) return fail(GPMPPI_E_INVALID, "batches do not split outputs (split must be 0)");
    if (t->split && t->groups != 1) return fail(GPMPPI_E_INVALID, "split outputs need groups = 1");
    if (batch) {
        if (t->wg_per_cu < 1 || t->wg_per_cu > wg_max)
            return fail(GPMPPI_E_INVALID, "wg_per_cu must lie in [1, %d] at this shape (got %d)", wg_max,
                        t->wg_per_cu);
        if (t->order != 0 && t->order != 1) return fail(GPMPPI_E_INVALID, "order must be 0 or 1");
    }
    return GPMPPI_OK;
}

// Rebuilds the item list and launch grid of a batch for a validated shape.
gpmppi_status batch_install(gpmppi_batch *b, const gpmppi_tuning &t) {
    const int B = 32 * t.groups;
    std::vector<std::pair<double, int2>> it;
    for (int p = 0; p < b->n; ++p) {
        const int K = b->ctx[p]->params.K;
        for (int blk = 0; blk < (K + B - 1) / B; ++blk) it.push_back({b->cost[p], make_int2(p, blk)});
    }
    if (t.order == 0)
        std::stable_sort(it.begin(), it.end(), [](const auto &a, const auto &c) { return a.first > c.first; });
    std::vector<int2> items;
    for (auto &e : it) items.push_back(e.second);
    for (int p = 0; p < b->n; ++p) b->ra_h[p].rotate = t.rotate;
    HIP_TRY(hipMemcpy(b->items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->ra, b->ra_h.data(), sizeof(RolloutArgs) * b->n, hipMemcpyHostToDevice));
    b->n_items = (int)items.size();
    b->G = t.groups;
    b->rotate = t.rotate;
    b->wg_per_cu = t.wg_per_cu;
    b->order = t.order;
    b->waves = t.waves;
    b->grid = std::max(1, std::min(b->n_items, b->cus * t.wg_per_cu));
    return GPMPPI_OK;
}

// Mean time in ms of reps launches of fn after one warm-up, on stream st.
template <typename F>
gpmppi_status time_launches(F &&fn, int reps, hipStream_t st, double &ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GPMPPI_E_HIP, "hipEventCreate failed");
    }
    gpmppi_status r = fn();
    if (r == GPMPPI_OK && hipEventRecord(e0, st) != hipSuccess) r = fail(GPMPPI_E_HIP, "hipEventRecord failed");
    for (int i = 0; i < reps && r == GPMPPI_OK; ++i) r = fn();
    if (r == GPMPPI_OK && hipEventRecord(e1, st) != hipSuccess) r = fail(GPMPPI_E_HIP, "hipEventRecord failed");
    float t = 0.0f;
    if (r == GPMPPI_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        r = fail(GPMPPI_E_HIP, "event timing failed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ms = (double)t / reps;
    return r;
}

}  // namespace

extern "C" {

gpmppi_status gpmppi_set_tuning(gpmppi_ctx *c, const gpmppi_tuning *t) {
    g_last_error.clear();
    if (!c) return fail(GPMPPI_E_INVALID, "ctx is NULL");
    gpmppi_status st = check_tuning(t, rollout_groups(c->params.precision, c->Mpad), 2, false);
    if (st != GPMPPI_OK) return st;
    if (t->split && !split_admissible(c, t->waves))
        return fail(GPMPPI_E_UNSUPPORTED, "split outputs: the doubled grid of %d workgroups does not fit the device at once",
                    2 * ((c->params.K + 31) / 32));
    if (t->waves == kPipeWaves && !rollout_pipe_admissible(c->params.precision, t->groups, c->Mpad))
        return fail(GPMPPI_E_UNSUPPORTED,
                    "waves = %d needs a BF16 form at M_pad = 1024 with the largest group count (here M_pad = %d)",
                    kPipeWaves, c->Mpad);
    c->groups = t->groups;
    c->rotate = t->rotate;
    c->waves = t->waves;
    c->split = t->split;
    return GPMPPI_OK;
}

gpmppi_status gpmppi_set_exchange_spin(gpmppi_ctx *c, int32_t polls) {
    g_last_error.clear();
    if (!c) return fail(GPMPPI_E_INVALID, "ctx is NULL");
    c->xspin = polls == 0 ? kXchSpin : (polls < 0 ? -1 : polls);
    return GPMPPI_OK;
}

gpmppi_status gpmppi_get_tuning(const gpmppi_ctx *c, gpmppi_tuning *t) {
    g_last_error.clear();
    if (!c || !t) return fail(GPMPPI_E_INVALID, "NULL argument");
    *t = gpmppi_tuning{c->groups, c->rotate, 1, 0, c->waves, c->split, 0.0};
    return GPMPPI_OK;
}

gpmppi_status gpmppi_tune(gpmppi_ctx *c, const float *x0_d, const float *U_d, uint64_t seed, int32_t reps,
                          gpmppi_tuning *chosen, void *stream) {
    g_last_error.clear();
    if (!c || !x0_d || !U_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (reps < 1 || reps > 100) return fail(GPMPPI_E_INVALID, "reps must lie in [1, 100] (got %d)", reps);
    hipStream_t st = (hipStream_t)stream;
    const int G_max = rollout_groups(c->params.precision, c->Mpad);
    const int keep_groups = c->groups, keep_rotate = c->rotate, keep_waves = c->waves, keep_split = c->split;
    gpmppi_tuning best{c->groups, c->rotate, 1, 0, c->waves, c->split, -1.0};
    for (int G = 1; G <= G_max; ++G)
        for (int rot = 0; rot <= 1; ++rot)
            for (int nw = 4; nw <= kPipeWaves; nw += 4) {
                // the wave-specialised shape walks W in one fixed order: rotate does not apply
                if (nw == kPipeWaves && (rot != 0 || !rollout_pipe_admissible(c->params.precision, G, c->Mpad)))
                    continue;
                for (int sp = 0; sp <= (G == 1 && nw != kPipeWaves && split_admissible(c, nw) ? 1 : 0); ++sp) {
                    c->groups = G;
                    c->rotate = rot;
                    c->waves = nw;
                    c->split = sp;
                    double ms = 0.0;
                    gpmppi_status r = time_launches(
                        [&]() { return gpmppi_rollout(c, x0_d, U_d, seed, c->cost_scratch, nullptr, stream); },
                        reps, st, ms);
                    if (r != GPMPPI_OK) {
                        c->groups = keep_groups;
                        c->rotate = keep_rotate;
                        c->waves = keep_waves;
                        c->split = keep_split;
                        return r;
                    }
                    if (best.ms < 0 || ms < best.ms) best = gpmppi_tuning{G, rot, 1, 0, nw, sp, ms};
                }
            }
    c->groups = best.groups;
    c->rotate = best.rotate;
    c->waves = best.waves;
    c->split = best.split;
    if (chosen) *chosen = best;
    return GPMPPI_OK;
}

gpmppi_status gpmppi_batch_init(int32_t n, const gpmppi_params params[], const gpmppi_gp gp[],
                                const gpmppi_obstacles obstacles[], const gpmppi_path paths[], gpmppi_batch **out) {
    g_last_error.clear();
    if (!out || !params || !gp || !obstacles || !paths) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n < 1 || n > 4096) return fail(GPMPPI_E_INVALID, "problem count must lie in [1, 4096]");
    for (int p = 0; p < n; ++p) {
        gpmppi_status st;
        if ((st = validate_params(&params[p])) != GPMPPI_OK) return st;
        if (params[p].precision != params[0].precision)
            return fail(GPMPPI_E_INVALID, "all problems of a batch need the same precision");
        if (params[p].tighten != 0)
            return fail(GPMPPI_E_UNSUPPORTED, "batches tighten along each sample's own covariance (tighten = 0)");
        if ((st = validate_gp(&gp[2 * p])) != GPMPPI_OK) return st;
        if ((st = validate_world(&obstacles[p], &paths[p])) != GPMPPI_OK) return st;
    }
    auto *b = new gpmppi_batch();
    b->n = n;
    b->precision = params[0].precision;
    b->U_off.assign(n + 1, 0);
    b->K_off.assign(n + 1, 0);
    for (int p = 0; p < n; ++p) {
        gpmppi_ctx *c = nullptr;
        gpmppi_status st = gpmppi_init(&params[p], &gp[2 * p], &obstacles[p], &paths[p], &c);
        if (st != GPMPPI_OK) {
            delete b;
            return st;
        }
        b->ctx.push_back(c);
        b->U_off[p + 1] = b->U_off[p] + 2LL * params[p].T;
        b->K_off[p + 1] = b->K_off[p] + params[p].K;
        b->Mpad_max = std::max(b->Mpad_max, c->Mpad);
        // one sample block's work: T steps of the triangular W walk, kernel vectors and world
        b->cost.push_back((double)params[p].T * ((double)c->Mpad * c->Mpad + 16.0 * c->Mpad +
                                                 (double)c->geo.P + 2.0 * c->n_obs + 200.0));
    }
    // every problem runs at the LDS plan of the largest M
    b->G_max = rollout_groups(b->precision, b->Mpad_max);
    long long max_items = 0, n_upd = 0;
    std::vector<int2> upd;
    for (int p = 0; p < n; ++p) {
        max_items += (params[p].K + 31) / 32;
        for (int k = 0; k < params[p].T; ++k) upd.push_back(make_int2(p, k));
    }
    n_upd = (long long)upd.size();
    b->n_upd = (int)n_upd;
    std::vector<UpdateArgs> ua(n);
    std::vector<int> T(n);
    std::vector<Dyn> dyn(n);
    b->ra_h.resize(n);
    for (int p = 0; p < n; ++p) {
        b->ra_h[p] = rollout_args(b->ctx[p], nullptr, nullptr, 0, nullptr, nullptr, nullptr);
        ua[p] = update_args(b->ctx[p], nullptr, nullptr, 0, nullptr, nullptr, nullptr);
        T[p] = params[p].T;
        dyn[p] = b->ctx[p]->dyn;
    }
    gpmppi_status st = GPMPPI_OK;
    auto track = [&](auto *p) {
        if (p) b->owned.push_back((void *)p);
        return p;
    };
    b->ra = track(dev_alloc<RolloutArgs>(n, st));
    b->ua = track(dev_alloc<UpdateArgs>(n, st));
    b->items = track(dev_alloc<int2>((size_t)max_items, st));
    b->upd_items = track(dev_alloc<int2>(upd.size(), st));
    b->U_off_d = track(dev_alloc<long long>(n + 1, st));
    b->K_off_d = track(dev_alloc<long long>(n + 1, st));
    b->T_d = track(dev_alloc<int>(n, st));
    b->dyn_d = track(dev_alloc<Dyn>(n, st));
    b->counters = track(dev_alloc<uint32_t>(4, st));
    b->cost_scratch = track(dev_alloc<float>((size_t)b->K_off[n], st));
    b->U_scratch = track(dev_alloc<float>((size_t)b->U_off[n], st));
    if (st != GPMPPI_OK) {
        delete b;
        return st;
    }
#define UP(dst, src, bytes)                                                                   \
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {                    \
        delete b;                                                                             \
        return fail(GPMPPI_E_HIP, "upload of the batch tables failed");                       \
    }
    UP(b->ua, ua.data(), sizeof(UpdateArgs) * n);
    UP(b->upd_items, upd.data(), sizeof(int2) * upd.size());
    UP(b->U_off_d, b->U_off.data(), sizeof(long long) * (n + 1));
    UP(b->K_off_d, b->K_off.data(), sizeof(long long) * (n + 1));
    UP(b->T_d, T.data(), sizeof(int) * n);
    UP(b->dyn_d, dyn.data(), sizeof(Dyn) * n);
#undef UP
    if (hipMemset(b->counters, 0, 4 * sizeof(uint32_t)) != hipSuccess) {
        delete b;
        return fail(GPMPPI_E_HIP, "hipMemset failed");
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
    b->cus = std::max(1, b->cus);
    b->wg_per_cu_max = wg_capacity(b->precision, b->G_max, b->Mpad_max);
    if ((st = batch_install(b, gpmppi_tuning{b->G_max, 1, b->wg_per_cu_max, 0, 4, 0, 0.0})) != GPMPPI_OK) {
        delete b;
        return st;
    }
    *out = b;
    return GPMPPI_OK;
}

gpmppi_status gpmppi_batch_set_tuning(gpmppi_batch *b, const gpmppi_tuning *t) {
    g_last_error.clear();
    if (!b) return fail(GPMPPI_E_INVALID, "batch is NULL");
    gpmppi_status st = check_tuning(t, b->G_max, t ? wg_capacity(b->precision, t->groups, b->Mpad_max) : 1, true);
    if (st != GPMPPI_OK) return st;
    return batch_install(b, *t);
}

gpmppi_status gpmppi_batch_get_tuning(const gpmppi_batch *b, gpmppi_tuning *t) {
    g_last_error.clear();
    if (!b || !t) return fail(GPMPPI_E_INVALID, "NULL argument");
    *t = gpmppi_tuning{b->G, b->rotate, b->wg_per_cu, b->order, b->waves, 0, 0.0};
    return GPMPPI_OK;
}

gpmppi_status gpmppi_batch_tune(gpmppi_batch *b, const float *x0_d, const float *U_d, uint64_t seed, int32_t reps,
                                gpmppi_tuning *chosen, void *stream) {
    g_last_error.clear();
    if (!b || !x0_d || !U_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (reps < 1 || reps > 100) return fail(GPMPPI_E_INVALID, "reps must lie in [1, 100] (got %d)", reps);
    hipStream_t st = (hipStream_t)stream;
    const gpmppi_tuning keep{b->G, b->rotate, b->wg_per_cu, b->order, b->waves, 0, 0.0};
    gpmppi_tuning best{0, 0, 0, 0, 4, 0, -1.0};
    for (int G = 1; G <= b->G_max; ++G) {
        const int wmax = wg_capacity(b->precision, G, b->Mpad_max);
        for (int rot = 0; rot <= 1; ++rot)
            for (int w = 1; w <= wmax; ++w)
                for (int ord = 0; ord <= 1; ++ord)
                for (int nw = 4; nw <= 8; nw += 4) {
                    const gpmppi_tuning cand{G, rot, w, ord, nw, 0, 0.0};
                    gpmppi_status r = batch_install(b, cand);
                    double ms = 0.0;
                    if (r == GPMPPI_OK) {
                        const BatchPtrs q{x0_d, U_d, b->U_scratch, b->cost_scratch, nullptr, seed, nullptr,
                                          b->U_off_d, b->K_off_d};
                        r = time_launches(
                            [&]() -> gpmppi_status {
                                HIP_TRY(launch_batch_patch(b->ra, b->ua, b->n, q, st));
                                HIP_TRY(launch_counter_reset(b->counters, st));
                                HIP_TRY(launch_rollout_batch(b->ra, b->items, b->n_items, b->counters,
                                                             b->precision, b->G, b->waves, b->Mpad_max, b->grid,
                                                             st));
                                return GPMPPI_OK;
                            },
                            reps, st, ms);
                    }
                    if (r != GPMPPI_OK) {
                        (void)batch_install(b, keep);
                        return r;
                    }
                    if (best.ms < 0 || ms < best.ms) best = gpmppi_tuning{G, rot, w, ord, nw, 0, ms};
                }
    }
    gpmppi_status r = batch_install(b, best);
    if (r != GPMPPI_OK) return r;
    if (chosen) *chosen = best;
    return GPMPPI_OK;
}

gpmppi_status gpmppi_batch_layout(const gpmppi_batch *b, int64_t *U_off, int64_t *K_off) {
    g_last_error.clear();
    if (!b) return fail(GPMPPI_E_INVALID, "batch is NULL");
    for (int p = 0; p <= b->n; ++p) {
        if (U_off) U_off[p] = b->U_off[p];
        if (K_off) K_off[p] = b->K_off[p];
    }
    return GPMPPI_OK;
}

gpmppi_status gpmppi_batch_step(gpmppi_batch *b, const float *x0_d, const float *U_d, uint64_t seed, float *U_out_d,
                                float *costs_d, float *weights_d, void *stream) {
    g_last_error.clear();
    if (!b || !x0_d || !U_d || !U_out_d || !costs_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const BatchPtrs q{x0_d, U_d, U_out_d, costs_d, weights_d, seed, nullptr, b->U_off_d, b->K_off_d};
    HIP_TRY(launch_batch_patch(b->ra, b->ua, b->n, q, st));
    return batch_enqueue_step(b, st);
}

gpmppi_status gpmppi_batch_closed_loop(gpmppi_batch *b, float *x_d, float *U_d, uint64_t seed0, int32_t n_steps,
                                       double amplitude, float *x_hist_d, int32_t use_graph, void *stream) {
    g_last_error.clear();
    if (!b || !x_d || !U_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (n_steps < 0) return fail(GPMPPI_E_INVALID, "n_steps must be >= 0");
    if (!is_fin(amplitude)) return fail(GPMPPI_E_NONFINITE, "non-finite plant amplitude");
    hipStream_t st = (hipStream_t)stream;
    uint32_t *step = b->counters + 1;
    HIP_TRY(launch_counter_reset(step, st));
    if (x_hist_d) HIP_TRY(hipMemcpyAsync(x_hist_d, x_d, sizeof(float) * 5 * b->n, hipMemcpyDeviceToDevice, st));
    const BatchPtrs q{x_d, U_d, U_d, b->cost_scratch, nullptr, seed0, step, b->U_off_d, b->K_off_d};
    HIP_TRY(launch_batch_patch(b->ra, b->ua, b->n, q, st));
    if (n_steps == 0) return GPMPPI_OK;
    auto enqueue = [&](hipStream_t s) -> gpmppi_status {
        gpmppi_status r = batch_enqueue_step(b, s);
        if (r != GPMPPI_OK) return r;
        HIP_TRY(launch_plant_shift_batch(x_d, U_d, b->U_off_d, b->T_d, b->dyn_d, (float)amplitude, step, x_hist_d,
                                         b->n, s));
        HIP_TRY(launch_counter_add(step, 1u, s));
        return GPMPPI_OK;
    };
    if (!use_graph) {
        for (int t = 0; t < n_steps; ++t) {
            gpmppi_status r = enqueue(st);
            if (r != GPMPPI_OK) return r;
        }
        return GPMPPI_OK;
    }
    return replay_captured(st, n_steps, enqueue);
}

void gpmppi_batch_destroy(gpmppi_batch *b) { delete b; }

double gpmppi_norm_quantile(double p) {
    if (!(p > 0.0 && p < 1.0)) return std::nan("");
    return norm_quantile(p);
}

// ------------------------------------------------------------------ differentiation form
}  // extern "C"

namespace {

// Pieces of the gradient's workspace (256-byte aligned offsets) for one call shape.
struct GradLayout {
    GradLaunch l{};
    int C = 1, nck = 1;
    int split = 0;   // two workgroups per 32 samples, one per GP output (when they fit the device at once)
    size_t o_ck = 0, o_seg = 0, o_R = 0, o_G = 0, o_b = 0, o_h = 0, o_u = 0, o_p = 0, o_bt = 0, o_c = 0;
    size_t o_x = 0, o_rp = 0;
    size_t bytes = 0;
};

// Validates a gradient call on the host and lays out its workspace.
gpmppi_status grad_check(const gpmppi_ctx *c, const float *x0_d, const float *U_d, double tau, int32_t checkpoint_every,
                         const float *J_d, const float *dU_d, const float *dlog_ell_d, const float *dlog_sf_d,
                         GradLayout &g) {
    if (!c || !x0_d || !U_d || !J_d || !dU_d || !dlog_ell_d || !dlog_sf_d) return fail(GPMPPI_E_INVALID, "NULL argument");
    if (!is_fin(tau) || !(tau > 0.0)) return fail(GPMPPI_E_INVALID, "tau must be finite and > 0");
    const int K = c->params.K, T = c->params.T, Mpad = c->Mpad;
    if (checkpoint_every < 1 || checkpoint_every > T)
        return fail(GPMPPI_E_INVALID, "checkpoint_every must lie in [1, T] (got %d)", checkpoint_every);
    if (!c->q32)
        return fail(GPMPPI_E_UNSUPPORTED, "the differentiation form supports M <= %d (padded M is %d)", kGradMaxMpad,
                    Mpad);
    if (c->n_terr > 0) return fail(GPMPPI_E_UNSUPPORTED, "the differentiation form has no terrain ensemble");
    if (c->params.tighten != 0 || c->params.w_goal != 0.0 || c->params.w_term != 0.0)
        return fail(GPMPPI_E_UNSUPPORTED, "the differentiation form has no goal terms or Step-2 tightening");
    g.C = checkpoint_every;
    GradLaunch &l = g.l;
    l.nwg = (K + 31) / 32;
    g.nck = (T + g.C - 1) / g.C;
    const int nb = (Mpad + 127) / 128;
    l.npairs = nb * (nb + 1) / 2;
    const long long TK = (long long)T * K;
    l.nsplit = (int)std::max(1LL, std::min<long long>({64LL, (512 + 2 * l.npairs - 1) / (2 * l.npairs), (TK + 1) / 2}));
    l.nbterm = (Mpad + kThreads - 1) / kThreads;
    size_t off = 0;
    auto take = [&](size_t nfloat) {
        const size_t at = off;
        off += (nfloat * sizeof(float) + 255) / 256 * 256;
        return at;
    };
    g.split = c->grad_split && 2 * l.nwg <= grad_split_capacity(Mpad) ? 1 : 0;
    g.o_ck = take((size_t)2 * g.nck * 20 * K);                  // one copy per role
    g.o_seg = take((size_t)l.nwg * 2 * (g.C + 1) * 28 * 32);    // per block and role
    g.o_R = take((size_t)2 * TK * Mpad);
    g.o_G = take((size_t)2 * TK);
    g.o_b = take((size_t)l.nwg * 2 * Mpad * 2);
    g.o_h = take((size_t)l.nwg * 10 * 2);
    g.o_u = take((size_t)l.nwg * T * 2);
    g.o_p = take((size_t)2 * l.npairs * l.nsplit * 4 * 2);
    g.o_bt = take((size_t)2 * l.nbterm * 4 * 2);
    g.o_c = take((size_t)K);
    g.o_x = take((size_t)l.nwg * kGradXchPerBlock * 2);         // 64-bit exchange records
    g.o_rp = take((size_t)l.nwg);
    g.bytes = off;
    return GPMPPI_OK;
}

// Enqueues the adjoint rollout and its reductions with the workspace at ws (device memory of at
// least g.bytes; no part of it needs to start at zero).
gpmppi_status grad_enqueue(const gpmppi_ctx *c, const GradLayout &g, char *ws, const float *x0_d, const float *U_d,
                           uint64_t seed, double tau, float *J_d, float *dU_d, float *dlog_ell_d, float *dlog_sf_d,
                           float *costs_d, hipStream_t stream) {
    GradLaunch l = g.l;
    GradArgs a{};
    a.gp = c->gp;
    a.geo = c->geo;
    a.cw = c->cw;
    a.dyn = c->dyn;
    a.noise = noise_of(c);
    a.noise.key0 = (uint32_t)seed;
    a.noise.key1 = (uint32_t)(seed >> 32);
    a.K = c->params.K;
    a.T = c->params.T;
    a.C = g.C;
    a.nck = g.nck;
    a.inv_tau = (float)(1.0 / tau);
    a.inv_K = 1.0f / (float)a.K;
    a.q32 = c->q32;
    a.q_stride = c->q_stride;
    a.x0 = x0_d;
    a.U = U_d;
    a.costs = costs_d ? costs_d : reinterpret_cast<float *>(ws + g.o_c);
    a.ckpt = reinterpret_cast<float *>(ws + g.o_ck);
    a.seg = reinterpret_cast<float *>(ws + g.o_seg);
    a.R = reinterpret_cast<float *>(ws + g.o_R);
    a.Gw = reinterpret_cast<float *>(ws + g.o_G);
    a.bpart = reinterpret_cast<double *>(ws + g.o_b);
    a.hpart = reinterpret_cast<double *>(ws + g.o_h);
    a.upart = reinterpret_cast<float *>(ws + g.o_u);
    l.ppart = reinterpret_cast<double *>(ws + g.o_p);
    l.bterm = reinterpret_cast<double *>(ws + g.o_bt);
    a.split = g.split;
    a.xrec = reinterpret_cast<unsigned long long *>(ws + g.o_x);
    a.repair = reinterpret_cast<uint32_t *>(ws + g.o_rp);
    a.xspin = c->xspin;
    a.flags = c->flags;
    l.J = J_d;
    l.dU = dU_d;
    l.dlog_ell = dlog_ell_d;
    l.dlog_sf = dlog_sf_d;
    HIP_TRY(launch_grad(a, l, stream));
    return GPMPPI_OK;
}

}  // namespace

extern "C" {

gpmppi_status gpmppi_grad(gpmppi_ctx *c, const float *x0_d, const float *U_d, uint64_t seed, double tau,
                          int32_t checkpoint_every, float *J_d, float *dU_d, float *dlog_ell_d, float *dlog_sf_d,
                          float *costs_d, void *stream) {
    g_last_error.clear();
    GradLayout g;
    gpmppi_status st = grad_check(c, x0_d, U_d, tau, checkpoint_every, J_d, dU_d, dlog_ell_d, dlog_sf_d, g);
    if (st != GPMPPI_OK) return st;
    if (g.bytes > c->grad_ws_bytes) {
        if (c->grad_ws) (void)hipFree(c->grad_ws);
        c->grad_ws = nullptr;
        c->grad_ws_bytes = 0;
        if (hipMalloc(&c->grad_ws, g.bytes) != hipSuccess) {
            c->grad_ws = nullptr;
            return fail(GPMPPI_E_NOMEM, "hipMalloc of the %zu-byte gradient workspace failed", g.bytes);
        }
        c->grad_ws_bytes = g.bytes;
    }
    return grad_enqueue(c, g, static_cast<char *>(c->grad_ws), x0_d, U_d, seed, tau, J_d, dU_d, dlog_ell_d,
                        dlog_sf_d, costs_d, (hipStream_t)stream);
}

gpmppi_status gpmppi_set_grad_split(gpmppi_ctx *c, int32_t split) {
    g_last_error.clear();
    if (!c) return fail(GPMPPI_E_INVALID, "ctx is NULL");
    if (split != 0 && split != 1) return fail(GPMPPI_E_INVALID, "split must be 0 or 1 (got %d)", split);
    c->grad_split = split;
    return GPMPPI_OK;
}

gpmppi_status gpmppi_grad_noalloc(gpmppi_ctx *c, const float *x0_d, const float *U_d, uint64_t seed, double tau,
                                  int32_t checkpoint_every, float *J_d, float *dU_d, float *dlog_ell_d,
                                  float *dlog_sf_d, float *costs_d, void *stream) {
    g_last_error.clear();
    GradLayout g;
    gpmppi_status st = grad_check(c, x0_d, U_d, tau, checkpoint_every, J_d, dU_d, dlog_ell_d, dlog_sf_d, g);
    if (st != GPMPPI_OK) return st;
    if (g.bytes > kScratchBytes)
        return fail(GPMPPI_E_NOMEM,
                    "the allocation-free gradient needs %zu bytes of scratch, more than its %zu-byte maximum "
                    "(about 8 T K M_pad bytes are needed; use gpmppi_grad)",
                    g.bytes, kScratchBytes);
    if (!c->scratch) return fail(GPMPPI_E_HIP, "the scratch array of this context's device has no address");
    return grad_enqueue(c, g, static_cast<char *>(c->scratch), x0_d, U_d, seed, tau, J_d, dU_d, dlog_ell_d,
                        dlog_sf_d, costs_d, (hipStream_t)stream);
}

void gpmppi_destroy(gpmppi_ctx *c) { delete c; }

}  // extern "C"
