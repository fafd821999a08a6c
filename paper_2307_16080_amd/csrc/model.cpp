// model.cpp -- the learned cost model: features of (problem, tile config),
// a small MLP trained on the GPU by the library's own kernels (mlp.hip) to
// predict log(time), and its use as a ranking for the tuner.
//
// The paper's tuning experiment (Sec. 4.3) searches the tile / unroll space
// with a black-box optimiser because no formal cost model of the hardware is
// at hand; here the measurements the tuner already takes train a model that
// ranks configurations, so later searches measure only the most promising.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "internal.hpp"

struct mlk_cost_model {
    int hidden = 64;
    int D0 = 0;
    std::vector<float> X;   // raw features, samples x D0
    std::vector<float> y;   // log(time in us)
    std::vector<float> mu, sd;  // feature normalisation
    float ymu = 0.f, ysd = 1.f;
    std::vector<float> params;  // host copy of the initial parameters, kMembers networks
    float* d_params = nullptr;  // kMembers parameter vectors back to back (as are d_m, d_v)
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_g = nullptr;
    float* d_loss = nullptr;
    int64_t step = 0;
    bool trained = false;
    uint64_t seed = 0;
};

namespace mlk {

namespace {

constexpr int kFeatures = 37;
// The model is a small ensemble: kMembers networks of the same shape, started
// from different initial weights and batch orders, whose log-time predictions
// are averaged (one network's ranking of close configurations varies with its
// initialisation more than the measurements it was trained on).
constexpr int kMembers = 3;

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
double lg(double v) { return std::log2(std::max(v, 1.0)); }

int64_t param_count(int D0, int H) { return (int64_t)D0 * H + H + (int64_t)H * H + H + H + 1; }

}  // namespace

int model_feature_count() { return kFeatures; }

void model_features(const Shape& s, const mlk_tile_config& c, int cus, float* f) {
    const int64_t M = std::max<int64_t>(s.M, 1), N = std::max<int64_t>(s.N, 1), K = std::max<int64_t>(s.K, 1);
    const int sk = std::max(1, c.split_k);
    const int64_t tm = cdiv(M, c.bm), tn = cdiv(N, c.bn);
    const int64_t tiles = tm * tn * sk;
    const int64_t stages = cdiv(cdiv(K, c.bk), sk);
    const int es = s.dt == DT_F32 ? 4 : s.dt == DT_BF16 ? 2 : 1;
    const int lds = 2 * (c.bm + c.bn) * (c.bk * es + 16);
    const int occ = lds > 80 * 1024 ? 1 : 2;
    const double waves = (double)tiles / ((double)cus * occ);
    int i = 0;
    f[i++] = (float)lg((double)M);
    f[i++] = (float)lg((double)N);
    f[i++] = (float)lg((double)K);
    f[i++] = (float)lg(c.bm);
    f[i++] = (float)lg(c.bn);
    f[i++] = (float)lg(c.bk);
    f[i++] = (float)c.wm;
    f[i++] = (float)c.wn;
    f[i++] = (float)lg(sk);
    f[i++] = c.group_m > 1 ? 1.f : 0.f;
    f[i++] = (float)c.xcd_remap;
    f[i++] = (float)lg((double)tiles);
    f[i++] = (float)std::min(waves, 64.0);
    f[i++] = (float)(waves - std::floor(waves));
    f[i++] = (float)((double)M / (double)(tm * c.bm));
    f[i++] = (float)((double)N / (double)(tn * c.bn));
    f[i++] = (float)((double)K / (double)(stages * sk * c.bk));
    f[i++] = (float)lg((double)stages);
    f[i++] = (float)lg((double)c.bm * c.bn / (c.bm + c.bn));
    f[i++] = (float)lds / 65536.f;
    f[i++] = s.conv ? 1.f : 0.f;
    f[i++] = s.dt == DT_F32 ? 1.f : 0.f;
    f[i++] = s.dt == DT_BF16 ? 1.f : 0.f;
    f[i++] = s.dt == DT_I8 ? 1.f : 0.f;
    f[i++] = s.dt == DT_F8 ? 1.f : 0.f;
    // work on the critical path: rounds of tiles times the work of one tile
    f[i++] = (float)lg(std::ceil(waves) * (double)c.bm * c.bn * c.bk * stages);
    f[i++] = (float)c.layout;
    // kernel family: register-staged (0), register-loaded direct layout (1),
    // direct-to-LDS ring (its depth)
    f[i++] = c.stages == 1 ? 1.f : 0.f;
    f[i++] = c.stages >= 2 ? (float)c.stages : 0.f;
    // convolution view (zero for a matmul): channels, filter taps and stride,
    // and the sizes the channels-last layout transposes before its GEMM (input,
    // and the filter unless it is 1 x 1)
    const double taps = s.conv ? (double)s.conv_kh * s.conv_kw : 0.0;
    const double in_el = s.conv ? (double)std::max<int64_t>(s.conv_in, 1) : 0.0;
    f[i++] = s.conv ? (float)lg((double)s.conv_c) : 0.f;
    f[i++] = (float)taps;
    f[i++] = s.conv ? (float)s.conv_sh : 0.f;
    f[i++] = (float)lg(in_el);
    f[i++] = c.layout == 1 ? (float)lg(in_el) : 0.f;
    f[i++] = c.layout == 1 && taps > 1 ? (float)lg((double)M * K) : 0.f;
    f[i++] = c.layout == 2 ? 1.f : 0.f;
    f[i++] = c.mfma == 32 ? 1.f : 0.f;  // 32 x 32 MFMA tiles
}

static mlk_status upload_params(mlk_cost_model* m) {
    const int64_t P = param_count(m->D0, m->hidden) * kMembers;
    hipError_t e = hipSuccess;
    if (!m->d_params) {
        if ((e = hipMalloc((void**)&m->d_params, sizeof(float) * P)) != hipSuccess ||
            (e = hipMalloc((void**)&m->d_m, sizeof(float) * P)) != hipSuccess ||
            (e = hipMalloc((void**)&m->d_v, sizeof(float) * P)) != hipSuccess ||
            (e = hipMalloc((void**)&m->d_g, sizeof(float) * P)) != hipSuccess ||
            (e = hipMalloc((void**)&m->d_loss, sizeof(float))) != hipSuccess)
            return hip_fail(e, "model allocation");
    }
    std::vector<float> zeros((size_t)P, 0.f);
    if ((e = hipMemcpy(m->d_params, m->params.data(), sizeof(float) * P, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(m->d_m, zeros.data(), sizeof(float) * P, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(m->d_v, zeros.data(), sizeof(float) * P, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "model upload");
    m->step = 0;
    return MLK_OK;
}

mlk_status model_predict_shape(mlk_cost_model* m, const Shape& s,
                               const std::vector<mlk_tile_config>& cfgs, std::vector<float>* us) {
    if (!m) return fail(MLK_ERR_NULL, "model is NULL");
    if (!m->trained) return fail(MLK_ERR_ARG, "model has not been trained");
    const int n = (int)cfgs.size();
    us->assign((size_t)n, 0.f);
    if (n == 0) return MLK_OK;
    const int D0 = m->D0;
    std::vector<float> X((size_t)n * D0);
    const int cus = device_cus();
    for (int i = 0; i < n; ++i) {
        model_features(s, cfgs[i], cus, &X[(size_t)i * D0]);
        for (int j = 0; j < D0; ++j) X[(size_t)i * D0 + j] = (X[(size_t)i * D0 + j] - m->mu[j]) / m->sd[j];
    }
    float *dX = nullptr, *dy = nullptr;
    hipError_t e;
    if ((e = hipMalloc((void**)&dX, sizeof(float) * X.size())) != hipSuccess) return hip_fail(e, "predict alloc");
    if ((e = hipMalloc((void**)&dy, sizeof(float) * n * kMembers)) != hipSuccess) {
        (void)hipFree(dX);
        return hip_fail(e, "predict alloc");
    }
    const int64_t P = param_count(D0, m->hidden);
    mlk_status st = MLK_OK;
    if ((e = hipMemcpy(dX, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice)) != hipSuccess)
        st = hip_fail(e, "predict upload");
    else {
        ScratchUse scratch;
        if ((st = scratch.begin(sizeof(float) * mlp_forward_words(n, m->hidden, m->hidden), 0, "model predict")) ==
            MLK_OK) {
            for (int k = 0; k < kMembers && e == hipSuccess; ++k)
                e = launch_mlp_forward(n, D0, m->hidden, m->hidden, m->d_params + k * P, dX, dy + (int64_t)k * n,
                                       (float*)scratch.ptr(), 0);
            st = scratch.end();
            if (e != hipSuccess) st = hip_fail(e, "predict forward");
        }
    }
    std::vector<float> all((size_t)n * kMembers);
    if (st == MLK_OK && e == hipSuccess) {
        if ((e = hipMemcpy(all.data(), dy, sizeof(float) * all.size(), hipMemcpyDeviceToHost)) != hipSuccess)
            st = hip_fail(e, "predict download");
    }
    (void)hipFree(dX);
    (void)hipFree(dy);
    if (st != MLK_OK) return st;
    // the members' normalised log-time predictions averaged, then back to microseconds
    for (int i = 0; i < n; ++i) {
        double a = 0.0;
        for (int k = 0; k < kMembers; ++k) a += all[(size_t)k * n + i];
        (*us)[i] = std::exp((float)(a / kMembers) * m->ysd + m->ymu);
    }
    return MLK_OK;
}

}  // namespace mlk

using namespace mlk;

extern "C" {

int32_t mlk_model_feature_count(void) { return kFeatures; }

mlk_status mlk_model_features(const mlk_problem* p, const mlk_tile_config* cfg, float* out) {
    clear_error();
    if (!cfg || !out) return fail(MLK_ERR_NULL, "features: NULL pointer");
    Shape s;
    mlk_status st = shape_of_problem(p, &s);
    if (st != MLK_OK) return st;
    model_features(s, *cfg, device_cus(), out);
    return MLK_OK;
}

mlk_status mlk_model_create(int32_t hidden, uint64_t seed, mlk_cost_model** out) {
    clear_error();
    if (!out) return fail(MLK_ERR_NULL, "model_create: out is NULL");
    if (hidden < 1 || hidden > 256) return fail(MLK_ERR_ARG, "model_create: hidden must be in [1, 256]");
    mlk_cost_model* m = new mlk_cost_model();
    m->hidden = hidden;
    m->D0 = kFeatures;
    m->seed = seed;
    // He-uniform initialisation of every member's weights, zero biases
    const int64_t P = param_count(m->D0, hidden);
    m->params.assign((size_t)(P * kMembers), 0.f);
    std::mt19937_64 rng(seed);
    const int64_t D0 = m->D0, H = hidden;
    for (int k = 0; k < kMembers; ++k) {
        auto fill = [&](int64_t off, int64_t fan_in, int64_t count) {
            const float lim = std::sqrt(6.0f / (float)fan_in);
            std::uniform_real_distribution<float> u(-lim, lim);
            for (int64_t i = 0; i < count; ++i) m->params[(size_t)(k * P + off + i)] = u(rng);
        };
        fill(0, D0, D0 * H);
        fill(D0 * H + H, H, H * H);
        fill(D0 * H + H + H * H + H, H, H);
    }
    mlk_status st = upload_params(m);
    if (st != MLK_OK) {
        mlk_model_destroy(m);
        return st;
    }
    *out = m;
    return MLK_OK;
}

void mlk_model_destroy(mlk_cost_model* m) {
    if (!m) return;
    for (float* p : {m->d_params, m->d_m, m->d_v, m->d_g, m->d_loss})
        if (p) (void)hipFree(p);
    delete m;
}

mlk_status mlk_model_add_sample(mlk_cost_model* m, const mlk_problem* p,
                                const mlk_tile_config* cfg, double time_us) {
    clear_error();
    if (!m || !cfg) return fail(MLK_ERR_NULL, "add_sample: NULL pointer");
    if (!(time_us > 0.0) || !std::isfinite(time_us)) return fail(MLK_ERR_ARG, "add_sample: time must be > 0");
    Shape s;
    mlk_status st = shape_of_problem(p, &s);
    if (st != MLK_OK) return st;
    std::vector<float> f((size_t)m->D0);
    model_features(s, *cfg, device_cus(), f.data());
    m->X.insert(m->X.end(), f.begin(), f.end());
    m->y.push_back((float)std::log(time_us));
    return MLK_OK;
}

int64_t mlk_model_sample_count(const mlk_cost_model* m) { return m ? (int64_t)m->y.size() : 0; }

mlk_status mlk_model_train(mlk_cost_model* m, int32_t epochs, int32_t batch, float lr,
                           float* final_loss) {
    clear_error();
    if (!m) return fail(MLK_ERR_NULL, "train: model is NULL");
    const int64_t n = (int64_t)m->y.size();
    if (n < 2) return fail(MLK_ERR_ARG, "train: need at least two samples");
    if (epochs < 1 || batch < 1 || !(lr > 0.f)) return fail(MLK_ERR_ARG, "train: bad epochs / batch / lr");
    const int D0 = m->D0, H = m->hidden;
    const int64_t P = param_count(D0, H);
    // normalisation statistics over the training set
    m->mu.assign(D0, 0.f);
    m->sd.assign(D0, 1.f);
    for (int j = 0; j < D0; ++j) {
        double a = 0, b = 0;
        for (int64_t i = 0; i < n; ++i) a += m->X[(size_t)(i * D0 + j)];
        a /= (double)n;
        for (int64_t i = 0; i < n; ++i) {
            const double d = m->X[(size_t)(i * D0 + j)] - a;
            b += d * d;
        }
        b = std::sqrt(b / (double)n);
        m->mu[j] = (float)a;
        m->sd[j] = b > 1e-6 ? (float)b : 1.f;
    }
    double a = 0, b = 0;
    for (float v : m->y) a += v;
    a /= (double)n;
    for (float v : m->y) b += (v - a) * (v - a);
    b = std::sqrt(b / (double)n);
    m->ymu = (float)a;
    m->ysd = b > 1e-6 ? (float)b : 1.f;

    std::vector<float> Xn((size_t)(n * D0)), yn((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < D0; ++j) Xn[(size_t)(i * D0 + j)] = (m->X[(size_t)(i * D0 + j)] - m->mu[j]) / m->sd[j];
        yn[(size_t)i] = (m->y[(size_t)i] - m->ymu) / m->ysd;
    }
    // restart from the initial weights so training is a function of the samples
    mlk_status st = upload_params(m);
    if (st != MLK_OK) return st;

    float *dX = nullptr, *dy = nullptr;
    hipError_t e;
    if ((e = hipMalloc((void**)&dX, sizeof(float) * Xn.size())) != hipSuccess) return hip_fail(e, "train alloc");
    if ((e = hipMalloc((void**)&dy, sizeof(float) * n)) != hipSuccess) {
        (void)hipFree(dX);
        return hip_fail(e, "train alloc");
    }
    // one workspace for every step (the full-batch loss at the end is the largest)
    ScratchUse scratch;
    if ((st = scratch.begin(sizeof(float) * mlp_loss_grad_words(n, H, H), 0, "model training")) != MLK_OK) {
        (void)hipFree(dX);
        (void)hipFree(dy);
        return st;
    }
    float* ws = (float*)scratch.ptr();
    std::vector<int64_t> perm((size_t)n);
    std::vector<float> Xs(Xn.size()), ys(yn.size());
    float loss = 0.f;
    st = MLK_OK;
    // each member: its own initial weights, Adam state and batch order
    for (int k = 0; k < kMembers && st == MLK_OK; ++k) {
        float* pk = m->d_params + k * P;
        float* mk = m->d_m + k * P;
        float* vk = m->d_v + k * P;
        std::iota(perm.begin(), perm.end(), 0);
        std::mt19937_64 rng((m->seed + 0x9E37ull * k) ^ 0xA5A5A5A5ull);
        int64_t step = 0;
        for (int ep = 0; ep < epochs && st == MLK_OK; ++ep) {
            std::shuffle(perm.begin(), perm.end(), rng);
            for (int64_t i = 0; i < n; ++i) {
                memcpy(&Xs[(size_t)(i * D0)], &Xn[(size_t)(perm[i] * D0)], sizeof(float) * D0);
                ys[(size_t)i] = yn[(size_t)perm[i]];
            }
            if ((e = hipMemcpy(dX, Xs.data(), sizeof(float) * Xs.size(), hipMemcpyHostToDevice)) != hipSuccess ||
                (e = hipMemcpy(dy, ys.data(), sizeof(float) * ys.size(), hipMemcpyHostToDevice)) != hipSuccess) {
                st = hip_fail(e, "train upload");
                break;
            }
            for (int64_t off = 0; off < n; off += batch) {
                const int64_t B = std::min<int64_t>(batch, n - off);
                if ((e = launch_mlp_loss_grad(B, D0, H, H, pk, dX + off * D0, dy + off, m->d_g, m->d_loss, ws,
                                              0)) != hipSuccess ||
                    (e = launch_adam(P, pk, m->d_g, mk, vk, lr, 0.9f, 0.999f, 1e-8f, ++step, 0)) != hipSuccess) {
                    st = hip_fail(e, "train step");
                    break;
                }
            }
        }
        m->step += step;
    }
    if (st == MLK_OK) {
        // full-batch loss of the final parameters, averaged over the members
        if ((e = hipMemcpy(dX, Xn.data(), sizeof(float) * Xn.size(), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(dy, yn.data(), sizeof(float) * yn.size(), hipMemcpyHostToDevice)) != hipSuccess)
            st = hip_fail(e, "train final loss");
        for (int k = 0; k < kMembers && st == MLK_OK; ++k) {
            float lk = 0.f;
            if ((e = launch_mlp_loss_grad(n, D0, H, H, m->d_params + k * P, dX, dy, m->d_g, m->d_loss, ws, 0)) !=
                    hipSuccess ||
                (e = hipMemcpy(&lk, m->d_loss, sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
                st = hip_fail(e, "train final loss");
            loss += lk / kMembers;
        }
    }
    const mlk_status rel = scratch.end();
    if (st == MLK_OK) st = rel;
    (void)hipFree(dX);
    (void)hipFree(dy);
    if (st != MLK_OK) return st;
    m->trained = true;
    if (final_loss) *final_loss = loss;
    return MLK_OK;
}

mlk_status mlk_model_predict(mlk_cost_model* m, const mlk_problem* p,
                             const mlk_tile_config* cfgs, int32_t n, float* pred_us) {
    clear_error();
    if (!m || !pred_us || (n > 0 && !cfgs)) return fail(MLK_ERR_NULL, "predict: NULL pointer");
    if (n < 0) return fail(MLK_ERR_ARG, "predict: n < 0");
    Shape s;
    mlk_status st = shape_of_problem(p, &s);
    if (st != MLK_OK) return st;
    std::vector<mlk_tile_config> v(cfgs, cfgs + n);
    std::vector<float> us;
    st = model_predict_shape(m, s, v, &us);
    if (st != MLK_OK) return st;
    std::copy(us.begin(), us.end(), pred_us);
    return MLK_OK;
}

}  // extern "C"
