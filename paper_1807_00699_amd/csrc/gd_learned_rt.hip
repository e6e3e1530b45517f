// C ABI of the learned proposal (kernels: gd_learned.hip; contracts: include/gd.h).
#include "gd_batch_rt.h"
#include "gd_internal.h"
#include "gd_learned.h"
#include "../../include/gd.h"

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace gd;

static_assert(GD_NFEAT == kMlpF, "feature count");
static_assert(GD_MLP_NPARAM == kMlpNParam, "parameter count");

struct gd_solver;   // defined in gd_runtime.hip
namespace gd {
BatchSolver *solver_batch(gd_solver *s);   // gd_runtime.hip
}

struct gd_mlp {
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    float *params = nullptr, *mom = nullptr, *vel = nullptr;
    int step = 0;
    // workspace for M rows
    int cap = 0;
    float *out = nullptr, *X = nullptr, *labels = nullptr;
    int *spin_inst = nullptr;
    int capK = 0;
    float *sigma = nullptr;
    int *seg = nullptr;
    float *partial = nullptr, *grad = nullptr;
    double *loss_part = nullptr, *loss = nullptr;
};

namespace {

// workgroups of the training step, each writing one gradient partial: one
// per compute unit of the GPU (a workgroup takes 87 KiB of the CU's 160 KiB
// of LDS, so one runs per CU)
constexpr int kParts = 256;

#define GD_TRY(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return gd_fail(e_ == hipErrorOutOfMemory ? GD_E_OOM : GD_E_DEVICE,           \
                           (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

template <class T>
hipError_t dm(T **p, size_t n) {
    return hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T));
}

void free_ws(gd_mlp *m) {
    void *ps[] = {m->out, m->X, m->labels, m->spin_inst};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    m->out = m->X = m->labels = nullptr;
    m->spin_inst = nullptr;
    m->cap = 0;
}

int ensure_ws(gd_mlp *m, int M, int K) {
    if (M > m->cap) {
        free_ws(m);
        if (dm(&m->out, (size_t)M * 2) || dm(&m->X, (size_t)M * kMlpF) || dm(&m->labels, M) ||
            dm(&m->spin_inst, M)) {
            free_ws(m);
            return gd_fail(GD_E_OOM, "MLP workspace allocation failed");
        }
        m->cap = M;
    }
    if (K + 1 > m->capK) {
        if (m->sigma) (void)hipFree(m->sigma);
        if (m->seg) (void)hipFree(m->seg);
        m->sigma = nullptr;
        m->seg = nullptr;
        if (dm(&m->sigma, K + 1) || dm(&m->seg, K + 1)) return gd_fail(GD_E_OOM, "MLP workspace allocation failed");
        m->capK = K + 1;
    }
    return GD_OK;
}

// He-normal initial weights (Box-Muller on SplitMix64 uniforms), zero biases
void init_params(std::vector<float> &p, uint64_t seed) {
    auto sm = [](uint64_t x) {
        x += 0x9E3779B97F4A7C15ull;
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        return x ^ (x >> 31);
    };
    auto uni = [&](uint64_t c) { return (double(sm(seed ^ sm(c)) >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    p.assign(kMlpNParam, 0.0f);
    const int F = kMlpF, H = kMlpH, O = kMlpOut;
    const int ranges[3][3] = {{0, F * H, F}, {F * H + H, H * H, H}, {F * H + H + H * H + H, H * O, H}};
    uint64_t c = 0;
    for (auto &r : ranges)
        for (int q = 0; q < r[1]; ++q, c += 2) {
            const double u1 = uni(c), u2 = uni(c + 1);
            const double z = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
            p[r[0] + q] = float(z * std::sqrt(2.0 / r[2]));
        }
}

hipMemcpyKind kind_in(const gd_mlp *m) {
    return (m->flags & GD_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}

}  // namespace

extern "C" {

int gd_mlp_create(gd_mlp **out, const float *params, uint64_t seed, uint32_t flags) {
    if (!out) return gd_fail(GD_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    gd_mlp *m = new (std::nothrow) gd_mlp();
    if (!m) return gd_fail(GD_E_OOM, "host allocation failed");
    m->flags = flags;
    if (dm(&m->params, kMlpNParam) || dm(&m->mom, kMlpNParam) || dm(&m->vel, kMlpNParam) ||
        dm(&m->partial, (size_t)kParts * kMlpNParam) || dm(&m->loss_part, kParts) || dm(&m->grad, kMlpNParam) ||
        dm(&m->loss, 1)) {
        gd_mlp_destroy(m);
        return gd_fail(GD_E_OOM, "MLP allocation failed");
    }
    if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
        gd_mlp_destroy(m);
        return gd_fail(GD_E_DEVICE, "hipStreamCreate failed");
    }
    int rc = gd_mlp_set_params(m, params);
    if (params == nullptr) {
        std::vector<float> p;
        init_params(p, seed);
        const uint32_t f = m->flags;
        m->flags &= ~GD_F_DEVICE_PTRS;
        rc = gd_mlp_set_params(m, p.data());
        m->flags = f;
    }
    if (rc != GD_OK) {
        gd_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return GD_OK;
}

void gd_mlp_destroy(gd_mlp *m) {
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    free_ws(m);
    void *ps[] = {m->params, m->mom, m->vel, m->partial, m->grad, m->loss_part, m->loss, m->sigma, m->seg};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    if (m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
}

int gd_mlp_set_params(gd_mlp *m, const float *params) {
    if (!m) return gd_fail(GD_E_INVALID_ARG, "mlp is NULL");
    if (params) {
        std::vector<float> h(kMlpNParam);
        if (m->flags & GD_F_DEVICE_PTRS) GD_TRY(hipMemcpy(h.data(), params, kMlpNParam * 4, hipMemcpyDeviceToHost));
        else std::memcpy(h.data(), params, kMlpNParam * 4);
        for (float v : h)
            if (!std::isfinite(v)) return gd_fail(GD_E_NONFINITE, "parameters are not finite");
        GD_TRY(hipMemcpy(m->params, h.data(), kMlpNParam * 4, hipMemcpyHostToDevice));
    }
    GD_TRY(hipMemset(m->mom, 0, kMlpNParam * 4));
    GD_TRY(hipMemset(m->vel, 0, kMlpNParam * 4));
    m->step = 0;
    return GD_OK;
}

int gd_mlp_get_params(gd_mlp *m, float *params) {
    if (!m || !params) return gd_fail(GD_E_INVALID_ARG, "NULL argument");
    GD_TRY(hipStreamSynchronize(m->stream));
    GD_TRY(hipMemcpy(params, m->params, kMlpNParam * 4,
                     (m->flags & GD_F_DEVICE_PTRS) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    return GD_OK;
}

int gd_mlp_forward(gd_mlp *m, int32_t M, const float *X, float *out, int32_t fp16) {
    if (!m || !X || !out || M < 0) return gd_fail(GD_E_INVALID_ARG, "bad argument");
    if (M == 0) return GD_OK;
    int rc = ensure_ws(m, M, 0);
    if (rc != GD_OK) return rc;
    const float *Xd = X;
    if (fp16 && (m->flags & GD_F_DEVICE_PTRS) && reinterpret_cast<uintptr_t>(X) % 16)
        return gd_fail(GD_E_INVALID_ARG, "X must be 16-byte aligned for the FP16 kernel");
    if (!(m->flags & GD_F_DEVICE_PTRS)) {
        GD_TRY(hipMemcpyAsync(m->X, X, (size_t)M * kMlpF * 4, hipMemcpyHostToDevice, m->stream));
        Xd = m->X;
    }
    float *od = (m->flags & GD_F_DEVICE_PTRS) ? out : m->out;
    GD_TRY(launch_mlp_forward(m->params, Xd, od, M, fp16 != 0, m->stream));
    if (!(m->flags & GD_F_DEVICE_PTRS))
        GD_TRY(hipMemcpyAsync(out, m->out, (size_t)M * 2 * 4, hipMemcpyDeviceToHost, m->stream));
    GD_TRY(hipStreamSynchronize(m->stream));
    return GD_OK;
}

int gd_mlp_train_step(gd_mlp *m, int32_t M, const float *X, const float *labels, int32_t K,
                      const int32_t *seg, float lr, double *loss, float *grad) {
    if (!m || !X || !labels || !seg || M < 1 || K < 1 || !(lr >= 0.0f))
        return gd_fail(GD_E_INVALID_ARG, "bad argument");
    if (seg[0] != 0 || seg[K] != M) return gd_fail(GD_E_INVALID_ARG, "seg must run from 0 to M");
    std::vector<int> inst((size_t)M);
    for (int k = 0; k < K; ++k) {
        if (seg[k + 1] <= seg[k]) return gd_fail(GD_E_INVALID_ARG, "empty or decreasing segment");
        for (int i = seg[k]; i < seg[k + 1]; ++i) inst[i] = k;
    }
    int rc = ensure_ws(m, M, K);
    if (rc != GD_OK) return rc;
    GD_TRY(hipMemcpyAsync(m->X, X, (size_t)M * kMlpF * 4, kind_in(m), m->stream));
    GD_TRY(hipMemcpyAsync(m->labels, labels, (size_t)M * 4, kind_in(m), m->stream));
    GD_TRY(hipMemcpyAsync(m->seg, seg, (size_t)(K + 1) * 4, hipMemcpyHostToDevice, m->stream));
    GD_TRY(hipMemcpyAsync(m->spin_inst, inst.data(), (size_t)M * 4, hipMemcpyHostToDevice, m->stream));
    if (lr > 0.0f) m->step += 1;
    MlpTrainArgs a{};
    a.params = m->params;
    a.mom = m->mom;
    a.vel = m->vel;
    a.X = m->X;
    a.labels = m->labels;
    a.seg = m->seg;
    a.spin_inst = m->spin_inst;
    a.M = M;
    a.out = m->out;
    a.sigma = m->sigma;
    a.partial = m->partial;
    a.loss_part = m->loss_part;
    a.grad_out = m->grad;
    a.loss = m->loss;
    GD_TRY(launch_mlp_train_step(a, K, kParts, lr, std::max(m->step, 1), m->stream));
    double L = 0.0;
    GD_TRY(hipMemcpyAsync(&L, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
    if (grad) GD_TRY(hipMemcpyAsync(grad, m->grad, kMlpNParam * 4, hipMemcpyDeviceToHost, m->stream));
    GD_TRY(hipStreamSynchronize(m->stream));
    if (loss) *loss = L;
    return GD_OK;
}

int gd_features(gd_solver *s, int32_t iters, float *feats, float *lambda, float *vecs) {
    if (!s || !feats || iters < 0) return gd_fail(GD_E_INVALID_ARG, "bad argument");
    BatchSolver *b = solver_batch(s);
    if (!b) return gd_fail(GD_E_UNSUPPORTED, "features are computed for batch solvers");
    BatchView v;
    batch_view(b, &v);
    if ((size_t)v.nmax * 16 * 4 > 160 * 1024) return gd_fail(GD_E_UNSUPPORTED, "instance too large for the feature kernel");
    float *df = nullptr, *dl = nullptr, *dv = nullptr;
    GD_TRY(dm(&df, (size_t)v.total * kMlpF));
    if (lambda) GD_TRY(dm(&dl, (size_t)v.K * 8));
    if (vecs) GD_TRY(dm(&dv, (size_t)v.total * 8));
    FeatArgs a{};
    a.inst_n = v.d_n;
    a.inst_spin = v.d_spin;
    a.inst_inv_s = v.d_inv_s;
    a.ell_idx = v.d_idx;
    a.ell_w = v.d_w;
    a.dmax = v.dmax;
    a.nmax = v.nmax;
    a.iters = iters;
    a.feats = df;
    a.lambda = dl;
    a.vecs = dv;
    hipError_t e = launch_features(a, v.K, v.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(feats, df, (size_t)v.total * kMlpF * 4, hipMemcpyDeviceToHost, v.stream);
    if (e == hipSuccess && lambda) e = hipMemcpyAsync(lambda, dl, (size_t)v.K * 32, hipMemcpyDeviceToHost, v.stream);
    if (e == hipSuccess && vecs) e = hipMemcpyAsync(vecs, dv, (size_t)v.total * 32, hipMemcpyDeviceToHost, v.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(v.stream);
    (void)hipFree(df);
    if (dl) (void)hipFree(dl);
    if (dv) (void)hipFree(dv);
    if (e != hipSuccess) return gd_fail(GD_E_DEVICE, hipGetErrorString(e));
    return GD_OK;
}

int gd_propose(gd_solver *s, gd_mlp *m, int32_t R, int32_t feat_iters, double alpha, double beta,
               uint64_t seed) {
    if (!s || !m || feat_iters < 0) return gd_fail(GD_E_INVALID_ARG, "bad argument");
    if (!(alpha >= 0.0 && alpha <= 1.0) || !std::isfinite(beta))
        return gd_fail(GD_E_INVALID_ARG, "alpha must be in [0, 1], beta finite");
    BatchSolver *b = solver_batch(s);
    if (!b) return gd_fail(GD_E_UNSUPPORTED, "proposals are made for batch solvers");
    int rc = batch_prepare_state(b, R);
    if (rc != GD_OK) return rc;
    BatchView v;
    batch_view(b, &v);
    if ((size_t)v.nmax * 16 * 4 > 160 * 1024) return gd_fail(GD_E_UNSUPPORTED, "instance too large for the feature kernel");
    float *df = nullptr, *dout = nullptr;
    GD_TRY(dm(&df, (size_t)v.total * kMlpF));
    hipError_t e = dm(&dout, (size_t)v.total * 2);
    FeatArgs a{};
    a.inst_n = v.d_n;
    a.inst_spin = v.d_spin;
    a.inst_inv_s = v.d_inv_s;
    a.ell_idx = v.d_idx;
    a.ell_w = v.d_w;
    a.dmax = v.dmax;
    a.nmax = v.nmax;
    a.iters = feat_iters;
    a.feats = df;
    if (e == hipSuccess) e = launch_features(a, v.K, v.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(v.stream);
    if (e == hipSuccess) e = launch_mlp_forward(m->params, df, dout, int(v.total), true, v.stream);
    ProposeArgs p{};
    p.inst_n = v.d_n;
    p.inst_spin = v.d_spin;
    p.inst_state = v.d_state;
    p.K = v.K;
    p.total_state = v.total * R;
    p.out = dout;
    p.x = v.d_x;
    p.gam = v.d_gam;
    p.eps = v.d_eps;
    p.seed = seed;
    p.amp = v.amp;
    p.alpha = alpha;
    p.beta = beta;
    p.eps0 = v.eps0;
    p.gamma0 = float(v.gamma0);
    if (e == hipSuccess) e = launch_propose(p, v.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(v.stream);
    (void)hipFree(df);
    if (dout) (void)hipFree(dout);
    if (e != hipSuccess) return gd_fail(GD_E_DEVICE, hipGetErrorString(e));
    return batch_finish_init(b);
}

}  // extern "C"
