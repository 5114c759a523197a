// costmodel.cpp -- host side of the learned cost model (C ABI). The network is
// d -> H (x layers) -> 1 with ReLU; parameters, gradients, Adam moments and
// activations live in caller-owned device memory; every arithmetic step runs
// in the kernels of kf_mlp.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <new>
#include <vector>

#include "kf_internal.h"

namespace kf {
hipError_t mlp_gemm(int M, int N, int K, const float* A, long sai, long sak, const float* B, long sbk, long sbj,
                    float* C, long ldc, const float* bias, int relu, const float* mask, long ldm, hipStream_t st);
hipError_t mlp_colsum(int M, int N, const float* dY, long ld, float* db, hipStream_t st);
hipError_t mlp_mse(int n, const float* p, const float* y, float* dp, float* loss, hipStream_t st);
hipError_t mlp_adam(long n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t st);
}  // namespace kf

using namespace kf;

struct kf_mlp {
    int d = 0, h = 0, L = 0;                 // input dim, hidden width, hidden layers
    std::vector<long> w_off, b_off, in_dim, out_dim;  // per layer (L + 1 layers)
    long nparams = 0;
};

namespace {

// Workspace: L activation buffers (n x h), prediction and its gradient (n),
// two gradient buffers (n x h), padded.
size_t ws_floats(const kf_mlp* m, long n) { return (size_t)(m->L + 2) * n * m->h + 2 * (size_t)n + 64; }

#define HIPCHK(x)                                                                     \
    do {                                                                              \
        hipError_t e__ = (x);                                                         \
        if (e__ != hipSuccess) return set_error(KF_ERR_HIP, hipGetErrorString(e__));  \
    } while (0)

kf_status forward(const kf_mlp* m, const float* P, const float* X, int n, float* ws, hipStream_t st) {
    const float* in = X;
    for (int l = 0; l < m->L; ++l) {
        float* H = ws + (size_t)l * n * m->h;
        HIPCHK(mlp_gemm(n, m->h, (int)m->in_dim[l], in, m->in_dim[l], 1, P + m->w_off[l], m->out_dim[l], 1, H, m->h,
                        P + m->b_off[l], 1, nullptr, 0, st));
        in = H;
    }
    float* pred = ws + (size_t)(m->L + 2) * n * m->h;
    const int l = m->L;
    HIPCHK(mlp_gemm(n, 1, m->h, in, m->h, 1, P + m->w_off[l], 1, 1, pred, 1, P + m->b_off[l], 0, nullptr, 0, st));
    return KF_OK;
}

}  // namespace

extern "C" {

kf_status kf_mlp_create(int32_t in_dim, int32_t hidden, int32_t layers, kf_mlp** out) {
    if (!out || in_dim < 1 || hidden < 1 || layers < 1 || in_dim > 4096 || hidden > 4096 || layers > 16)
        return set_error(KF_ERR_ARG, "bad MLP dimensions");
    auto* m = new kf_mlp();
    m->d = in_dim;
    m->h = hidden;
    m->L = layers;
    long off = 0;
    for (int l = 0; l <= layers; ++l) {
        long i = l == 0 ? in_dim : hidden, o = l == layers ? 1 : hidden;
        m->in_dim.push_back(i);
        m->out_dim.push_back(o);
        m->w_off.push_back(off);
        off += i * o;
        m->b_off.push_back(off);
        off += o;
    }
    m->nparams = off;
    *out = m;
    return KF_OK;
}

void kf_mlp_destroy(kf_mlp* m) { delete m; }

kf_status kf_mlp_param_count(const kf_mlp* m, int64_t* n) {
    if (!m || !n) return set_error(KF_ERR_ARG, "null argument");
    *n = m->nparams;
    return KF_OK;
}

kf_status kf_mlp_layout(const kf_mlp* m, int32_t layer, int64_t* w_off, int64_t* b_off, int64_t* rows, int64_t* cols) {
    if (!m || layer < 0 || layer > m->L) return set_error(KF_ERR_ARG, "bad layer");
    if (w_off) *w_off = m->w_off[layer];
    if (b_off) *b_off = m->b_off[layer];
    if (rows) *rows = m->in_dim[layer];
    if (cols) *cols = m->out_dim[layer];
    return KF_OK;
}

kf_status kf_mlp_init_params(const kf_mlp* m, uint64_t seed, float* host_params) {
    if (!m || !host_params) return set_error(KF_ERR_ARG, "null argument");
    // He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)) from SplitMix64; zero biases.
    uint64_t state = seed * 0x9E3779B97F4A7C15ULL + 0xD1B54A32D192ED03ULL;
    auto next = [&]() {
        uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    std::memset(host_params, 0, sizeof(float) * (size_t)m->nparams);
    for (int l = 0; l <= m->L; ++l) {
        const double bound = std::sqrt(6.0 / (double)m->in_dim[l]);
        for (long i = 0; i < m->in_dim[l] * m->out_dim[l]; ++i) {
            double u = (double)(next() >> 11) * (1.0 / 9007199254740992.0);
            host_params[m->w_off[l] + i] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    return KF_OK;
}

kf_status kf_mlp_workspace_bytes(const kf_mlp* m, int32_t batch, size_t* bytes) {
    if (!m || !bytes || batch < 1) return set_error(KF_ERR_ARG, "bad argument");
    *bytes = ws_floats(m, batch) * sizeof(float);
    return KF_OK;
}

kf_status kf_mlp_forward(const kf_mlp* m, const float* params, const float* X, int32_t n, float* pred, void* ws,
                         size_t ws_bytes, void* stream) {
    if (!m || !params || !X || !pred || !ws || n < 1) return set_error(KF_ERR_ARG, "bad argument");
    if (ws_bytes < ws_floats(m, n) * sizeof(float)) return set_error(KF_ERR_WORKSPACE, "MLP workspace too small");
    hipStream_t st = (hipStream_t)stream;
    float* w = (float*)ws;
    kf_status s = forward(m, params, X, n, w, st);
    if (s != KF_OK) return s;
    const float* p = w + (size_t)(m->L + 2) * n * m->h;
    HIPCHK(hipMemcpyAsync(pred, p, sizeof(float) * (size_t)n, hipMemcpyDeviceToDevice, st));
    return KF_OK;
}

kf_status kf_mlp_loss_grad(const kf_mlp* m, const float* params, const float* X, const float* y, int32_t n,
                           float* grads, float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (!m || !params || !X || !y || !grads || !ws || n < 1) return set_error(KF_ERR_ARG, "bad argument");
    if (ws_bytes < ws_floats(m, n) * sizeof(float)) return set_error(KF_ERR_WORKSPACE, "MLP workspace too small");
    hipStream_t st = (hipStream_t)stream;
    float* w = (float*)ws;
    kf_status s = forward(m, params, X, n, w, st);
    if (s != KF_OK) return s;
    const int h = m->h, L = m->L;
    float* pred = w + (size_t)(L + 2) * n * h;
    float* dpred = pred + n;
    float* g0 = w + (size_t)L * n * h;        // two n x h gradient buffers
    float* g1 = g0 + (size_t)n * h;
    auto H = [&](int l) -> const float* { return l == 0 ? X : w + (size_t)(l - 1) * n * h; };  // input of layer l
    HIPCHK(mlp_mse(n, pred, y, dpred, loss, st));
    // output layer: dW = H_L^T dpred, db = sum dpred, dH_L = dpred W^T masked by H_L > 0
    HIPCHK(mlp_gemm(h, 1, n, H(L), 1, h, dpred, 1, 1, grads + m->w_off[L], 1, nullptr, 0, nullptr, 0, st));
    HIPCHK(mlp_colsum(n, 1, dpred, 1, grads + m->b_off[L], st));
    HIPCHK(mlp_gemm(n, h, 1, dpred, 1, 1, params + m->w_off[L], 1, 1, g0, h, nullptr, 0, H(L), h, st));
    float* cur = g0;
    float* nxt = g1;
    for (int l = L - 1; l >= 0; --l) {
        const long in = m->in_dim[l];
        HIPCHK(mlp_gemm((int)in, h, n, H(l), 1, in, cur, h, 1, grads + m->w_off[l], h, nullptr, 0, nullptr, 0, st));
        HIPCHK(mlp_colsum(n, h, cur, h, grads + m->b_off[l], st));
        if (l > 0) {
            HIPCHK(mlp_gemm(n, h, h, cur, h, 1, params + m->w_off[l], 1, h, nxt, h, nullptr, 0, H(l), h, st));
            float* t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    return KF_OK;
}

kf_status kf_mlp_adam(const kf_mlp* m, float* params, const float* grads, float* mstate, float* vstate, int32_t step,
                      float lr, float beta1, float beta2, float eps, void* stream) {
    if (!m || !params || !grads || !mstate || !vstate || step < 1) return set_error(KF_ERR_ARG, "bad argument");
    const float c1 = 1.f - (float)std::pow((double)beta1, step);
    const float c2 = 1.f - (float)std::pow((double)beta2, step);
    HIPCHK(mlp_adam(m->nparams, params, grads, mstate, vstate, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream));
    return KF_OK;
}

}  // extern "C"

// ---- the cost model object: network, normalisation, and the caller's memory
namespace kf {
hipError_t mlp_col_stats(long n, int d, const float* X, float floor, float* mu, float* sd, hipStream_t st);
hipError_t mlp_gather_std(int rows, int d, const float* X, const int* idx, long row0, const float* mu,
                          const float* sd, float* out, hipStream_t st);
hipError_t mlp_unstd(int n, const float* p, const float* mu, const float* sd, float* out, hipStream_t st);
}  // namespace kf

// Parts of the bound device memory, each at a 256-byte boundary (offsets in
// bytes): parameters, gradients, Adam moments, the MLP workspace for `rows`
// rows, standardised features and targets, raw features staged from the
// host, predictions, minibatch row indices, and the statistics (feature means
// and deviations, target mean and deviation, the last loss).
struct CmLayout {
    size_t params, grads, mom1, mom2, ws, x, raw, y, out, idx, stats, total;
    size_t ws_floats;
};

struct kf_costmodel {
    kf_mlp* m = nullptr;
    uint64_t seed = 0;
    std::vector<float> params;        // host copy; authoritative while unbound
    std::vector<float> mu, sd;
    double y_mu = 0.0, y_sd = 1.0;
    float launch_us = 0.f;
    char* mem = nullptr;              // caller-owned device memory (kf_costmodel_bind)
    int64_t rows_cap = 0;
    CmLayout lay{};
    ~kf_costmodel() {
        if (m) kf_mlp_destroy(m);
    }
    float* f(size_t off) const { return (float*)(mem + off); }
};

namespace {

const int kPredictChunk = 8192;

CmLayout cm_layout(const kf_mlp* m, int64_t rows) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    CmLayout L{};
    const size_t pb = up((size_t)m->nparams * 4), d = (size_t)m->d, r = (size_t)rows;
    size_t o = 0;
    L.params = o; o += pb;
    L.grads = o; o += pb;
    L.mom1 = o; o += pb;
    L.mom2 = o; o += pb;
    L.ws_floats = ws_floats(m, rows);
    L.ws = o; o += up(L.ws_floats * 4);
    L.x = o; o += up(r * d * 4);
    L.raw = o; o += up(r * d * 4);
    L.y = o; o += up(r * 4);
    L.out = o; o += up(r * 4);
    L.idx = o; o += up(r * 4);
    L.stats = o; o += up((2 * d + 4) * 4);
    L.total = o;
    return L;
}

// Device copies of the statistics: mu[d], sd[d], y_mu, y_sd, loss.
float* st_mu(const kf_costmodel* cm) { return cm->f(cm->lay.stats); }
float* st_sd(const kf_costmodel* cm) { return st_mu(cm) + cm->m->d; }
float* st_ymu(const kf_costmodel* cm) { return st_mu(cm) + 2 * cm->m->d; }
float* st_ysd(const kf_costmodel* cm) { return st_ymu(cm) + 1; }
float* st_loss(const kf_costmodel* cm) { return st_ymu(cm) + 2; }

kf_status upload_state(kf_costmodel* cm, hipStream_t st) {
    const int d = cm->m->d;
    std::vector<float> stats(2 * d + 2);
    std::copy(cm->mu.begin(), cm->mu.end(), stats.begin());
    std::copy(cm->sd.begin(), cm->sd.end(), stats.begin() + d);
    stats[2 * d] = (float)cm->y_mu;
    stats[2 * d + 1] = (float)cm->y_sd;
    HIPCHK(hipMemcpyAsync(cm->f(cm->lay.params), cm->params.data(), cm->params.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(st_mu(cm), stats.data(), stats.size() * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return KF_OK;
}

kf_status need_bound(const kf_costmodel* cm, int64_t rows) {
    if (!cm->mem) return set_error(KF_ERR_UNBOUND, "the cost model has no device memory: kf_costmodel_bind first");
    if (rows > cm->rows_cap)
        return set_error(KF_ERR_WORKSPACE, "the bound cost-model memory holds fewer rows than this call needs");
    return KF_OK;
}

uint64_t splitmix(uint64_t& state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// log_us[0..c) of standardised feature rows at cm->lay.x (device) into dst (device).
kf_status predict_staged(kf_costmodel* cm, int c, float* dst, hipStream_t st) {
    float* ws = cm->f(cm->lay.ws);
    kf_status s = kf_mlp_forward(cm->m, cm->f(cm->lay.params), cm->f(cm->lay.x), c, cm->f(cm->lay.out), ws,
                                 cm->lay.ws_floats * 4, st);
    if (s != KF_OK) return s;
    HIPCHK(mlp_unstd(c, cm->f(cm->lay.out), st_ymu(cm), st_ysd(cm), dst, st));
    return KF_OK;
}

}  // namespace

extern "C" {

kf_status kf_costmodel_create(int32_t hidden, int32_t layers, uint64_t seed, kf_costmodel** out) {
    if (!out) return set_error(KF_ERR_ARG, "null argument");
    auto* cm = new (std::nothrow) kf_costmodel();
    if (!cm) return set_error(KF_ERR_NOMEM, "host allocation failed");
    std::unique_ptr<kf_costmodel> guard(cm);
    kf_status s = kf_mlp_create(KF_FEATURE_DIM, hidden, layers, &cm->m);
    if (s != KF_OK) return s;
    cm->seed = seed;
    cm->mu.assign(KF_FEATURE_DIM, 0.f);
    cm->sd.assign(KF_FEATURE_DIM, 1.f);
    cm->params.assign((size_t)cm->m->nparams, 0.f);
    kf_mlp_init_params(cm->m, seed, cm->params.data());
    *out = guard.release();
    return KF_OK;
}

void kf_costmodel_destroy(kf_costmodel* cm) { delete cm; }

kf_status kf_costmodel_workspace_bytes(const kf_costmodel* cm, int64_t rows, size_t* bytes) {
    if (!cm || !bytes || rows < 1 || rows > ((int64_t)1 << 24)) return set_error(KF_ERR_ARG, "bad argument");
    *bytes = cm_layout(cm->m, rows).total;
    return KF_OK;
}

kf_status kf_costmodel_bind(kf_costmodel* cm, void* mem, size_t bytes, int64_t rows, void* stream) {
    if (!cm || !mem || rows < 1 || rows > ((int64_t)1 << 24)) return set_error(KF_ERR_ARG, "bad argument");
    if ((uintptr_t)mem % 256) return set_error(KF_ERR_ALIGN, "cost-model memory must be 256-byte aligned");
    const CmLayout L = cm_layout(cm->m, rows);
    if (bytes < L.total) return set_error(KF_ERR_WORKSPACE, "cost-model memory smaller than kf_costmodel_workspace_bytes");
    if (cm->mem) {   // keep what training did in the memory bound before
        HIPCHK(hipStreamSynchronize((hipStream_t)stream));
        HIPCHK(hipMemcpy(cm->params.data(), cm->f(cm->lay.params), cm->params.size() * 4, hipMemcpyDeviceToHost));
    }
    cm->mem = (char*)mem;
    cm->rows_cap = rows;
    cm->lay = L;
    kf_status s = upload_state(cm, (hipStream_t)stream);
    if (s != KF_OK) cm->mem = nullptr;
    return s;
}

kf_status kf_costmodel_train(kf_costmodel* cm, const float* X, const float* y_log_us, int64_t n, int32_t epochs,
                             int32_t batch, float lr, uint64_t seed, void* stream, float* loss_per_epoch) {
    if (!cm || !X || !y_log_us || n < 2 || n > INT32_MAX || epochs < 1 || batch < 1 || !(lr > 0.f))
        return set_error(KF_ERR_ARG, "bad argument");
    kf_status s = need_bound(cm, batch);
    if (s != KF_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int d = cm->m->d;
    // feature and target standardisation from the training data (on the GPU)
    HIPCHK(mlp_col_stats(n, d, X, 1e-3f, st_mu(cm), st_sd(cm), st));
    HIPCHK(mlp_col_stats(n, 1, y_log_us, 1e-6f, st_ymu(cm), st_ysd(cm), st));
    std::vector<float> stats(2 * d + 2);
    HIPCHK(hipMemcpyAsync(stats.data(), st_mu(cm), stats.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    cm->mu.assign(stats.begin(), stats.begin() + d);
    cm->sd.assign(stats.begin() + d, stats.begin() + 2 * d);
    cm->y_mu = stats[2 * d];
    cm->y_sd = stats[2 * d + 1];
    const size_t pb = (size_t)cm->m->nparams * sizeof(float);
    HIPCHK(hipMemsetAsync(cm->f(cm->lay.mom1), 0, pb, st));
    HIPCHK(hipMemsetAsync(cm->f(cm->lay.mom2), 0, pb, st));
    std::vector<int32_t> perm((size_t)n);
    int* d_idx = (int*)(cm->mem + cm->lay.idx);
    uint64_t rng = seed * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
    int step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(splitmix(rng) % (uint64_t)(i + 1))]);
        double tot = 0.0;
        int cnt = 0;
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int b = (int)std::min<int64_t>(batch, n - b0);
            ++step;
            // the minibatch's rows, gathered and standardised on the GPU
            HIPCHK(hipMemcpyAsync(d_idx, perm.data() + b0, (size_t)b * 4, hipMemcpyHostToDevice, st));
            HIPCHK(mlp_gather_std(b, d, X, d_idx, 0, st_mu(cm), st_sd(cm), cm->f(cm->lay.x), st));
            HIPCHK(mlp_gather_std(b, 1, y_log_us, d_idx, 0, st_ymu(cm), st_ysd(cm), cm->f(cm->lay.y), st));
            s = kf_mlp_loss_grad(cm->m, cm->f(cm->lay.params), cm->f(cm->lay.x), cm->f(cm->lay.y), b,
                                 cm->f(cm->lay.grads), st_loss(cm), cm->f(cm->lay.ws), cm->lay.ws_floats * 4, stream);
            if (s != KF_OK) return s;
            s = kf_mlp_adam(cm->m, cm->f(cm->lay.params), cm->f(cm->lay.grads), cm->f(cm->lay.mom1),
                            cm->f(cm->lay.mom2), step, lr, 0.9f, 0.999f, 1e-8f, stream);
            if (s != KF_OK) return s;
            float l = 0.f;
            HIPCHK(hipMemcpyAsync(&l, st_loss(cm), sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            tot += l;
            ++cnt;
        }
        if (loss_per_epoch) loss_per_epoch[ep] = (float)(tot / std::max(cnt, 1));
    }
    return KF_OK;
}

kf_status kf_costmodel_predict(kf_costmodel* cm, const float* X, int64_t n, float* log_us, void* stream) {
    if (!cm || (n > 0 && (!X || !log_us)) || n < 0) return set_error(KF_ERR_ARG, "bad argument");
    kf_status s = need_bound(cm, 1);
    if (s != KF_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int d = cm->m->d;
    for (int64_t c0 = 0; c0 < n; c0 += cm->rows_cap) {
        const int c = (int)std::min<int64_t>(cm->rows_cap, n - c0);
        HIPCHK(mlp_gather_std(c, d, X, nullptr, c0, st_mu(cm), st_sd(cm), cm->f(cm->lay.x), st));
        s = predict_staged(cm, c, log_us + c0, st);
        if (s != KF_OK) return s;
    }
    return KF_OK;
}

kf_status kf_costmodel_plan_us(kf_costmodel* cm, const float* feats, int64_t rows, const int64_t* start,
                               int32_t nplans, double* us, void* stream) {
    if (!cm || nplans < 0 || rows < 0 || (nplans > 0 && (!start || !us)) || (rows > 0 && !feats))
        return set_error(KF_ERR_ARG, "bad argument");
    for (int32_t i = 0; i < nplans; ++i)
        if (start[i] < 0 || start[i] > start[i + 1] || start[i + 1] > rows)
            return set_error(KF_ERR_ARG, "plan row ranges must be ordered and inside the feature rows");
    kf_status s = need_bound(cm, 1);
    if (s != KF_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const int d = cm->m->d;
    std::vector<float> lg((size_t)rows);
    for (int64_t c0 = 0; c0 < rows; c0 += cm->rows_cap) {
        const int c = (int)std::min<int64_t>(cm->rows_cap, rows - c0);
        HIPCHK(hipMemcpyAsync(cm->f(cm->lay.raw), feats + c0 * d, (size_t)c * d * 4, hipMemcpyHostToDevice, st));
        HIPCHK(mlp_gather_std(c, d, cm->f(cm->lay.raw), nullptr, 0, st_mu(cm), st_sd(cm), cm->f(cm->lay.x), st));
        s = predict_staged(cm, c, cm->f(cm->lay.out), st);
        if (s != KF_OK) return s;
        HIPCHK(hipMemcpyAsync(lg.data() + c0, cm->f(cm->lay.out), (size_t)c * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    for (int32_t i = 0; i < nplans; ++i) {
        double t = 0.0;
        for (int64_t r = start[i]; r < start[i + 1]; ++r)
            t += std::exp((double)lg[r]) + (double)cm->launch_us * feats[r * d + 25];
        us[i] = t;
    }
    return KF_OK;
}

kf_status kf_costmodel_set_launch_us(kf_costmodel* cm, float us) {
    if (!cm || !(us >= 0.f)) return set_error(KF_ERR_ARG, "bad argument");
    cm->launch_us = us;
    return KF_OK;
}

kf_status kf_costmodel_get(const kf_costmodel* cm, float* params, float* mu, float* sd, double* y_mu_sd,
                           float* launch_us) {
    if (!cm) return set_error(KF_ERR_ARG, "null model");
    if (params) {
        if (cm->mem) {
            if (hipDeviceSynchronize() != hipSuccess ||
                hipMemcpy(params, cm->f(cm->lay.params), (size_t)cm->m->nparams * sizeof(float),
                          hipMemcpyDeviceToHost) != hipSuccess)
                return set_error(KF_ERR_HIP, "reading the model parameters failed");
        } else {
            std::memcpy(params, cm->params.data(), cm->params.size() * sizeof(float));
        }
    }
    if (mu) std::memcpy(mu, cm->mu.data(), cm->mu.size() * sizeof(float));
    if (sd) std::memcpy(sd, cm->sd.data(), cm->sd.size() * sizeof(float));
    if (y_mu_sd) { y_mu_sd[0] = cm->y_mu; y_mu_sd[1] = cm->y_sd; }
    if (launch_us) *launch_us = cm->launch_us;
    return KF_OK;
}

kf_status kf_costmodel_set(kf_costmodel* cm, const float* params, const float* mu, const float* sd,
                           const double* y_mu_sd, float launch_us) {
    if (!cm || !params || !mu || !sd || !y_mu_sd || !(y_mu_sd[1] > 0.0)) return set_error(KF_ERR_ARG, "bad argument");
    for (int j = 0; j < cm->m->d; ++j)
        if (!(sd[j] > 0.f)) return set_error(KF_ERR_ARG, "feature scales must be positive");
    cm->params.assign(params, params + cm->m->nparams);
    cm->mu.assign(mu, mu + cm->m->d);
    cm->sd.assign(sd, sd + cm->m->d);
    cm->y_mu = y_mu_sd[0];
    cm->y_sd = y_mu_sd[1];
    cm->launch_us = launch_us;
    if (cm->mem) {
        if (hipDeviceSynchronize() != hipSuccess) return set_error(KF_ERR_HIP, "hipDeviceSynchronize failed");
        return upload_state(cm, nullptr);
    }
    return KF_OK;
}

// File: "KFCM" magic, int32 version 2, int32 feature dim, hidden, layers,
// int64 parameter count, float mu[d], sd[d], double y_mu, y_sd, float
// launch_us, float params[], then the FNV-1a 64 hash of everything after the
// magic; little-endian, as the host writes them. load checks magic, version,
// sizes and hash before it touches the GPU.
namespace {
uint64_t fnv64(const char* p, size_t n) {
    uint64_t h = 1469598103934665603ULL;
    for (size_t i = 0; i < n; ++i) {
        h ^= (unsigned char)p[i];
        h *= 1099511628211ULL;
    }
    return h;
}
void put_bytes(std::string& b, const void* v, size_t bytes) { b.append(static_cast<const char*>(v), bytes); }
}  // namespace

kf_status kf_costmodel_save(const kf_costmodel* cm, const char* path) {
    if (!cm || !path) return set_error(KF_ERR_ARG, "null argument");
    std::vector<float> p((size_t)cm->m->nparams);
    kf_status s = kf_costmodel_get(cm, p.data(), nullptr, nullptr, nullptr, nullptr);
    if (s != KF_OK) return s;
    std::string b;
    const int32_t hdr[4] = {2, cm->m->d, cm->m->h, cm->m->L};
    const int64_t np = cm->m->nparams;
    const double y[2] = {cm->y_mu, cm->y_sd};
    put_bytes(b, hdr, 16);
    put_bytes(b, &np, 8);
    put_bytes(b, cm->mu.data(), 4 * cm->mu.size());
    put_bytes(b, cm->sd.data(), 4 * cm->sd.size());
    put_bytes(b, y, 16);
    put_bytes(b, &cm->launch_us, 4);
    put_bytes(b, p.data(), 4 * p.size());
    const uint64_t h = fnv64(b.data(), b.size());
    FILE* f = std::fopen(path, "wb");
    if (!f) return set_error(KF_ERR_ARG, std::string("cannot write ") + path);
    bool ok = std::fwrite("KFCM", 1, 4, f) == 4 && std::fwrite(b.data(), 1, b.size(), f) == b.size() &&
              std::fwrite(&h, 8, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? KF_OK : set_error(KF_ERR_ARG, std::string("write failed: ") + path);
}

kf_status kf_costmodel_load(const char* path, kf_costmodel** out) {
    if (!path || !out) return set_error(KF_ERR_ARG, "null argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return set_error(KF_ERR_ARG, std::string("cannot read ") + path);
    std::string d;
    char buf[1 << 16];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) d.append(buf, got);
    std::fclose(f);
    const std::string bad = std::string("not a valid cost-model file of this library: ") + path;
    const size_t head = 4 + 16 + 8;
    if (d.size() < head + 8 || d.compare(0, 4, "KFCM") != 0) return set_error(KF_ERR_ARG, bad);
    int32_t hdr[4];
    int64_t np = 0;
    std::memcpy(hdr, d.data() + 4, 16);
    std::memcpy(&np, d.data() + 20, 8);
    if (hdr[0] != 2 || hdr[1] != KF_FEATURE_DIM || hdr[2] < 1 || hdr[2] > 4096 || hdr[3] < 1 || hdr[3] > 16 ||
        np < 1 || np > (int64_t)1 << 28)
        return set_error(KF_ERR_ARG, bad);
    const size_t body = head + 8 * (size_t)KF_FEATURE_DIM + 16 + 4 + 4 * (size_t)np;
    if (d.size() != body + 8) return set_error(KF_ERR_ARG, bad);
    uint64_t h = 0;
    std::memcpy(&h, d.data() + body, 8);
    if (fnv64(d.data() + 4, body - 4) != h) return set_error(KF_ERR_ARG, bad + " (checksum)");
    std::vector<float> mu(KF_FEATURE_DIM), sd(KF_FEATURE_DIM), p((size_t)np);
    double y[2];
    float lu = 0.f;
    size_t o = head;
    std::memcpy(mu.data(), d.data() + o, 4 * mu.size()); o += 4 * mu.size();
    std::memcpy(sd.data(), d.data() + o, 4 * sd.size()); o += 4 * sd.size();
    std::memcpy(y, d.data() + o, 16); o += 16;
    std::memcpy(&lu, d.data() + o, 4); o += 4;
    std::memcpy(p.data(), d.data() + o, 4 * p.size());
    kf_costmodel* cm = nullptr;
    kf_status s = kf_costmodel_create(hdr[2], hdr[3], 0, &cm);
    if (s != KF_OK) return s;
    std::unique_ptr<kf_costmodel> guard(cm);
    if (cm->m->nparams != np) return set_error(KF_ERR_ARG, bad);
    s = kf_costmodel_set(cm, p.data(), mu.data(), sd.data(), y, lu);
    if (s != KF_OK) return s;
    *out = guard.release();
    return KF_OK;
}

kf_status kf_costmodel_dims(const kf_costmodel* cm, int32_t* hidden, int32_t* layers, int64_t* nparams) {
    if (!cm) return set_error(KF_ERR_ARG, "null model");
    if (hidden) *hidden = cm->m->h;
    if (layers) *layers = cm->m->L;
    if (nparams) *nparams = cm->m->nparams;
    return KF_OK;
}

}  // extern "C"

namespace kf {
// Predicted times (us) of plans given as per-kernel feature rows: plan i owns
// rows [start[i], start[i + 1]); time = sum exp(prediction) + launch_us * launches.
kf_status costmodel_plan_us(kf_costmodel* cm, const std::vector<float>& feats, const std::vector<size_t>& start,
                            hipStream_t st, std::vector<double>* us) {
    const size_t rows = feats.size() / KF_FEATURE_DIM;
    std::vector<int64_t> st64(start.begin(), start.end());
    us->assign(start.size() - 1, 0.0);
    return kf_costmodel_plan_us(cm, feats.data(), (int64_t)rows, st64.data(), (int32_t)(start.size() - 1), us->data(),
                                st);
}
}  // namespace kf
