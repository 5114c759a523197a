// costmodel.cpp -- host side of the learned cost model (C ABI). The network is
// d -> H (x layers) -> 1 with ReLU; parameters, gradients, Adam moments and
// activations live in caller-owned device memory; every arithmetic step runs
// in the kernels of kf_mlp.hip.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
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
