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

// ---- the cost model object: network, its device state and the normalisation
struct kf_costmodel {
    kf_mlp* m = nullptr;
    uint64_t seed = 0;
    float* d_params = nullptr;
    float* d_grads = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    float* d_ws = nullptr;
    float* d_x = nullptr;
    float* d_y = nullptr;
    float* d_out = nullptr;
    size_t ws_cap = 0;   // floats of d_ws
    long rows_cap = 0;   // rows of d_x, d_y, d_out
    std::vector<float> mu, sd;
    double y_mu = 0.0, y_sd = 1.0;
    float launch_us = 0.f;
    ~kf_costmodel() {
        for (float* p : {d_params, d_grads, d_m, d_v, d_ws, d_x, d_y, d_out})
            if (p) (void)hipFree(p);
        if (m) kf_mlp_destroy(m);
    }
};

namespace {

const int kPredictChunk = 8192;

kf_status cm_reserve(kf_costmodel* cm, long rows) {
    if (rows <= cm->rows_cap) return KF_OK;
    for (float** p : {&cm->d_ws, &cm->d_x, &cm->d_y, &cm->d_out})
        if (*p) { (void)hipFree(*p); *p = nullptr; }
    cm->ws_cap = ws_floats(cm->m, rows);
    HIPCHK(hipMalloc((void**)&cm->d_ws, cm->ws_cap * sizeof(float)));
    HIPCHK(hipMalloc((void**)&cm->d_x, (size_t)rows * cm->m->d * sizeof(float)));
    HIPCHK(hipMalloc((void**)&cm->d_y, (size_t)rows * sizeof(float)));
    HIPCHK(hipMalloc((void**)&cm->d_out, (size_t)rows * sizeof(float)));
    cm->rows_cap = rows;
    return KF_OK;
}

uint64_t splitmix(uint64_t& state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
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
    std::vector<float> p((size_t)cm->m->nparams);
    kf_mlp_init_params(cm->m, seed, p.data());
    const size_t pb = p.size() * sizeof(float);
    for (float** d : {&cm->d_params, &cm->d_grads, &cm->d_m, &cm->d_v})
        HIPCHK(hipMalloc((void**)d, pb));
    HIPCHK(hipMemcpy(cm->d_params, p.data(), pb, hipMemcpyHostToDevice));
    *out = guard.release();
    return KF_OK;
}

void kf_costmodel_destroy(kf_costmodel* cm) { delete cm; }

kf_status kf_costmodel_train(kf_costmodel* cm, const float* X, const float* y_log_us, int64_t n, int32_t epochs,
                             int32_t batch, float lr, uint64_t seed, void* stream, float* loss_per_epoch) {
    if (!cm || !X || !y_log_us || n < 2 || epochs < 1 || batch < 1 || !(lr > 0.f))
        return set_error(KF_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const int d = cm->m->d;
    // feature and target standardisation from the training data
    std::vector<double> mu(d, 0.0), var(d, 0.0);
    double ym = 0.0, yv = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < d; ++j) mu[j] += X[i * d + j];
        ym += y_log_us[i];
    }
    for (int j = 0; j < d; ++j) mu[j] /= (double)n;
    ym /= (double)n;
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < d; ++j) var[j] += (X[i * d + j] - mu[j]) * (X[i * d + j] - mu[j]);
        yv += (y_log_us[i] - ym) * (y_log_us[i] - ym);
    }
    for (int j = 0; j < d; ++j) {
        cm->mu[j] = (float)mu[j];
        cm->sd[j] = (float)std::max(std::sqrt(var[j] / (double)n), 1e-3);
    }
    cm->y_mu = ym;
    cm->y_sd = std::max(std::sqrt(yv / (double)n), 1e-6);
    kf_status s = cm_reserve(cm, std::max<long>(batch, n));
    if (s != KF_OK) return s;
    const size_t pb = (size_t)cm->m->nparams * sizeof(float);
    HIPCHK(hipMemsetAsync(cm->d_m, 0, pb, st));
    HIPCHK(hipMemsetAsync(cm->d_v, 0, pb, st));
    std::vector<int64_t> perm(n);
    std::vector<float> xs((size_t)n * d), ys(n);
    uint64_t rng = seed * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
    int step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t i = 0; i < n; ++i) perm[i] = i;
        for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(int64_t)(splitmix(rng) % (uint64_t)(i + 1))]);
        for (int64_t i = 0; i < n; ++i) {
            const float* src = X + perm[i] * d;
            for (int j = 0; j < d; ++j) xs[i * d + j] = (src[j] - cm->mu[j]) / cm->sd[j];
            ys[i] = (float)((y_log_us[perm[i]] - cm->y_mu) / cm->y_sd);
        }
        HIPCHK(hipMemcpyAsync(cm->d_x, xs.data(), xs.size() * sizeof(float), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(cm->d_y, ys.data(), ys.size() * sizeof(float), hipMemcpyHostToDevice, st));
        double tot = 0.0;
        int cnt = 0;
        for (int64_t b0 = 0; b0 < n; b0 += batch) {
            const int b = (int)std::min<int64_t>(batch, n - b0);
            ++step;
            s = kf_mlp_loss_grad(cm->m, cm->d_params, cm->d_x + b0 * d, cm->d_y + b0, b, cm->d_grads, cm->d_out,
                                 cm->d_ws, cm->ws_cap * sizeof(float), stream);
            if (s != KF_OK) return s;
            s = kf_mlp_adam(cm->m, cm->d_params, cm->d_grads, cm->d_m, cm->d_v, step, lr, 0.9f, 0.999f, 1e-8f, stream);
            if (s != KF_OK) return s;
            float l = 0.f;
            HIPCHK(hipMemcpyAsync(&l, cm->d_out, sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            tot += l;
            ++cnt;
        }
        if (loss_per_epoch) loss_per_epoch[ep] = (float)(tot / std::max(cnt, 1));
    }
    return KF_OK;
}

kf_status kf_costmodel_predict(kf_costmodel* cm, const float* X, int64_t n, float* log_us, void* stream) {
    if (!cm || !X || !log_us || n < 0) return set_error(KF_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const int d = cm->m->d;
    kf_status s = cm_reserve(cm, kPredictChunk);
    if (s != KF_OK) return s;
    std::vector<float> xs((size_t)kPredictChunk * d), out(kPredictChunk);
    for (int64_t c0 = 0; c0 < n; c0 += kPredictChunk) {
        const int c = (int)std::min<int64_t>(kPredictChunk, n - c0);
        for (int64_t i = 0; i < c; ++i)
            for (int j = 0; j < d; ++j) xs[i * d + j] = (X[(c0 + i) * d + j] - cm->mu[j]) / cm->sd[j];
        HIPCHK(hipMemcpyAsync(cm->d_x, xs.data(), (size_t)c * d * sizeof(float), hipMemcpyHostToDevice, st));
        s = kf_mlp_forward(cm->m, cm->d_params, cm->d_x, c, cm->d_out, cm->d_ws, cm->ws_cap * sizeof(float), stream);
        if (s != KF_OK) return s;
        HIPCHK(hipMemcpyAsync(out.data(), cm->d_out, (size_t)c * sizeof(float), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int i = 0; i < c; ++i) log_us[c0 + i] = (float)(out[i] * cm->y_sd + cm->y_mu);
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
    if (params && hipMemcpy(params, cm->d_params, (size_t)cm->m->nparams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(KF_ERR_HIP, "reading the model parameters failed");
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
    if (hipMemcpy(cm->d_params, params, (size_t)cm->m->nparams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return set_error(KF_ERR_HIP, "writing the model parameters failed");
    cm->mu.assign(mu, mu + cm->m->d);
    cm->sd.assign(sd, sd + cm->m->d);
    cm->y_mu = y_mu_sd[0];
    cm->y_sd = y_mu_sd[1];
    cm->launch_us = launch_us;
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
    std::vector<float> lg(rows);
    kf_status s = kf_costmodel_predict(cm, feats.data(), (int64_t)rows, lg.data(), st);
    if (s != KF_OK) return s;
    us->assign(start.size() - 1, 0.0);
    for (size_t i = 0; i + 1 < start.size(); ++i)
        for (size_t r = start[i]; r < start[i + 1]; ++r)
            (*us)[i] += std::exp((double)lg[r]) + cm->launch_us * feats[r * KF_FEATURE_DIM + 25];
    return KF_OK;
}
}  // namespace kf
