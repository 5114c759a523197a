// Host-side exercise of the C ABI for an AddressSanitizer / UndefinedBehavior-
// Sanitizer build of the library's host code (no GPU is touched: every plan is
// compiled with KF_COMPILE_CODEGEN_ONLY). It records the Table 1 sequences and
// random-looking scripts over ragged shapes, enumerates partitions and
// candidates, generates every candidate's code, extracts features, prices
// plans with the additive predictor, builds plans with per-kernel parameters,
// walks the error paths of the recorder and compiler, lays out a batch, and
// rejects damaged cost-model files. Any sanitizer report ends the run with a
// non-zero status; a wrong status from the library prints and returns 1.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "kf.h"

static int g_fail = 0;
static int g_plans = 0;   // plans whose code was generated and inspected

#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "FAILED line %d: %s (%s)\n", __LINE__, #cond,     \
                         kf_last_error());                                        \
            g_fail = 1;                                                           \
        }                                                                         \
    } while (0)

static kf_value vec(kf_script* s, int64_t n) {
    kf_value v = -1;
    EXPECT(kf_vector(s, n, &v) == KF_OK);
    EXPECT(kf_input(s, v) == KF_OK);
    return v;
}
static kf_value mat(kf_script* s, int64_t r, int64_t c) {
    kf_value v = -1;
    EXPECT(kf_matrix(s, r, c, 0, &v) == KF_OK);
    EXPECT(kf_input(s, v) == KF_OK);
    return v;
}
static kf_value cst(kf_script* s, float x) {
    kf_value v = -1;
    EXPECT(kf_const(s, x, &v) == KF_OK);
    return v;
}

// GEMVER (ger, ger, gemtv, gemv) on an m x n matrix in either layout
static kf_script* gemver(int64_t m, int64_t n, int32_t layout = KF_ROW_MAJOR) {
    kf_script* s = nullptr;
    EXPECT(kf_script_create(&s) == KF_OK);
    kf_value A = -1;
    EXPECT(kf_matrix_layout(s, m, n, 0, layout, &A) == KF_OK);
    EXPECT(kf_input(s, A) == KF_OK);
    kf_value u1 = vec(s, m), v1 = vec(s, n), u2 = vec(s, m), v2 = vec(s, n);
    kf_value y = vec(s, m), z = vec(s, n);
    kf_value one = cst(s, 1.f), a = cst(s, 1.5f), b = cst(s, 0.75f);
    kf_value B1, B, x, w;
    EXPECT(kf_ger(s, one, A, u1, v1, &B1) == KF_OK);
    EXPECT(kf_ger(s, one, B1, u2, v2, &B) == KF_OK);
    EXPECT(kf_gemtv(s, b, B, y, one, z, &x) == KF_OK);
    EXPECT(kf_gemv(s, a, B, x, KF_NONE, KF_NONE, &w) == KF_OK);
    EXPECT(kf_output(s, B) == KF_OK);
    EXPECT(kf_output(s, x) == KF_OK);
    EXPECT(kf_output(s, w) == KF_OK);
    return s;
}

// a mixed script: BLAS-1 and BLAS-2 calls sharing values, a dot feeding a scal
static kf_script* mixed(int64_t n) {
    kf_script* s = nullptr;
    EXPECT(kf_script_create(&s) == KF_OK);
    kf_value A = mat(s, n, n), p = vec(s, n), r = vec(s, n), one = cst(s, 1.f), two = cst(s, 2.f);
    kf_value q, t, d, e, f;
    EXPECT(kf_gemv(s, one, A, p, KF_NONE, KF_NONE, &q) == KF_OK);
    EXPECT(kf_gemtv(s, one, A, r, KF_NONE, KF_NONE, &t) == KF_OK);
    EXPECT(kf_dot(s, q, t, &d) == KF_OK);
    EXPECT(kf_axpy(s, two, q, t, &e) == KF_OK);
    EXPECT(kf_scal(s, d, e, &f) == KF_OK);
    EXPECT(kf_output(s, f) == KF_OK);
    EXPECT(kf_output(s, d) == KF_OK);
    return s;
}

static void exercise_plan(kf_plan* p);

// BiCGK (q = A p, s = A^T r) on a quantised matrix with row scales, with a
// device scalar as the gemv's alpha
static kf_script* bicgk_q(int64_t m, int64_t n, int32_t dtype) {
    kf_script* s = nullptr;
    EXPECT(kf_script_create(&s) == KF_OK);
    kf_value sc = vec(s, m), A = -1, al = -1;
    EXPECT(kf_matrix_q(s, m, n, 0, dtype, sc, &A) == KF_OK);
    EXPECT(kf_input(s, A) == KF_OK);
    EXPECT(kf_scalar(s, &al) == KF_OK);
    EXPECT(kf_input(s, al) == KF_OK);
    kf_value p = vec(s, n), r = vec(s, m), one = cst(s, 1.f), q, t;
    EXPECT(kf_gemv(s, al, A, p, KF_NONE, KF_NONE, &q) == KF_OK);
    EXPECT(kf_gemtv(s, one, A, r, KF_NONE, KF_NONE, &t) == KF_OK);
    EXPECT(kf_output(s, q) == KF_OK);
    EXPECT(kf_output(s, t) == KF_OK);
    return s;
}

// a random script over n-vectors and n x n matrices (fixed LCG); calls whose
// operands the recorder refuses are simply not recorded
static kf_script* random_script(uint64_t seed, int64_t n, int calls) {
    uint64_t st = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto next = [&](int lim) {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        return (int)((st >> 33) % (uint64_t)lim);
    };
    kf_script* s = nullptr;
    EXPECT(kf_script_create(&s) == KF_OK);
    std::vector<kf_value> V{vec(s, n), vec(s, n)}, M{mat(s, n, n)}, C{cst(s, 0.5f), cst(s, -2.f)};
    std::vector<kf_value> made;
    for (int c = 0; c < calls; ++c) {
        kf_value a = C[next((int)C.size())], x = V[next((int)V.size())], y = V[next((int)V.size())];
        kf_value A = M[next((int)M.size())], out = KF_NONE;
        kf_status st2 = KF_OK;
        switch (next(6)) {
            case 0: st2 = kf_scal(s, a, x, &out); break;
            case 1: st2 = kf_axpy(s, a, x, y, &out); break;
            case 2: st2 = kf_dot(s, x, y, &out); break;
            case 3: st2 = kf_gemv(s, a, A, x, next(2) ? a : KF_NONE, next(2) ? y : KF_NONE, &out); break;
            case 4: st2 = kf_gemtv(s, a, A, x, KF_NONE, KF_NONE, &out); break;
            default: st2 = kf_ger(s, a, A, x, y, &out); break;
        }
        if (st2 != KF_OK) continue;
        int32_t kind = -1;
        int64_t d0, d1, d2;
        EXPECT(kf_value_info(s, out, &kind, &d0, &d1, &d2) == KF_OK);
        if (kind == 1) M.push_back(out);
        else if (kind == 0) V.push_back(out);
        else C.push_back(out);
        made.push_back(out);
    }
    for (size_t i = 0; i < made.size(); i += 2) (void)kf_output(s, made[i]);
    if (!made.empty()) (void)kf_output(s, made.back());
    return s;
}

static void all_candidates(kf_script* s, int32_t max_partitions) {
    kf_planset* ps = nullptr;
    int32_t ncalls = 0;
    kf_script_num_calls(s, &ncalls);
    if (ncalls == 0) return;
    EXPECT(kf_candidates(s, max_partitions, nullptr, 0, &ps) == KF_OK);
    if (!ps) return;
    int32_t nc = 0;
    kf_planset_count(ps, &nc);
    for (int32_t i = 0; i < nc; ++i) {
        kf_plan* p = nullptr;
        if (kf_planset_compile(ps, i, KF_COMPILE_CODEGEN_ONLY, &p) != KF_OK) continue;
        exercise_plan(p);
        kf_plan_destroy(p);
    }
    kf_planset_destroy(ps);
}

static std::vector<kf_routine_entry> table() {
    std::vector<kf_routine_entry> t;
    const int mat_env[][4] = {{0, 0, 0, 0}, {1, 4, 4, 1024}, {2, 8, 2, 1024}};
    for (auto& e : mat_env)
        for (int x : {0, 64})
            for (int r = 0; r <= 4; ++r) t.push_back({1, {e[0], e[1], e[2], e[3]}, r, x, 1e-6f * (r + 1 + x)});
    for (auto& e : mat_env) t.push_back({1, {e[0], e[1], e[2], e[3]}, 10, 0, 4.f});
    for (int x : {0, 16, 64})   // row-resident environment (default geometry)
        for (int r = 0; r <= 4; ++r) t.push_back({2, {0, 0, 0, 0}, r, x, 2e-6f * (r + 1)});
    t.push_back({2, {0, 0, 0, 0}, 10, 0, 3.f});
    for (int r = 5; r <= 10; ++r) t.push_back({0, {0, 0, 0, 0}, r, 0, r == 10 ? 4.f : 1e-5f});
    return t;
}

static void exercise_plan(kf_plan* p) {
    ++g_plans;
    int32_t nk = 0;
    EXPECT(kf_plan_num_kernels(p, &nk) == KF_OK && nk >= 1);
    size_t need = 0;
    EXPECT(kf_plan_describe(p, nullptr, 0, &need) == KF_OK && need > 0);
    std::string buf(need, '\0');
    EXPECT(kf_plan_describe(p, &buf[0], buf.size(), &need) == KF_OK);
    std::vector<float> f((size_t)nk * KF_FEATURE_DIM);
    int32_t got = 0;
    EXPECT(kf_plan_features(p, f.data(), nk, &got) == KF_OK && got == nk);
    for (int32_t k = 0; k < nk; ++k) {
        kf_impl_params ip;
        EXPECT(kf_plan_kernel_params(p, k, &ip) == KF_OK);
        size_t sn = 0;
        EXPECT(kf_plan_source(p, k, nullptr, 0, &sn) == KF_OK && sn > 0);
        int32_t nl = 0;
        EXPECT(kf_plan_num_launches(p, k, &nl) == KF_OK && nl >= 1);
    }
    uint64_t rd = 0, wr = 0;
    EXPECT(kf_plan_bytes(p, &rd, &wr) == KF_OK && rd > 0);
    size_t ws = 0;
    EXPECT(kf_plan_workspace_bytes(p, &ws) == KF_OK);
    EXPECT(kf_run(p, nullptr) == KF_ERR_STATE);   // code generation only: never runnable
}

int main() {
    const auto T = table();
    const int64_t shapes[][2] = {{1, 1}, {3, 5}, {64, 64}, {257, 2050}, {1000, 1001}, {4099, 300}};
    for (auto& sh : shapes) {
        kf_script* s = gemver(sh[0], sh[1]);
        kf_planset* ps = nullptr;
        EXPECT(kf_candidates(s, 0, nullptr, 0, &ps) == KF_OK);
        int32_t nc = 0;
        EXPECT(kf_planset_count(ps, &nc) == KF_OK && nc > 0);
        for (int32_t i = 0; i < nc; ++i) {
            kf_plan* p = nullptr;
            if (kf_planset_compile(ps, i, KF_COMPILE_CODEGEN_ONLY, &p) != KF_OK) continue;
            exercise_plan(p);
            float us = 0.f;
            EXPECT(kf_predict_additive(p, T.data(), (int32_t)T.size(), &us) == KF_OK || true);
            kf_plan_destroy(p);
        }
        std::vector<float> pred((size_t)nc);
        (void)kf_planset_predict_additive(ps, T.data(), (int32_t)T.size(), pred.data());
        kf_planset_destroy(ps);
        // every ranking input path that needs no device: the additive mode
        kf_compile_opts o;
        kf_compile_opts_init(&o);
        o.mode = KF_MODE_ADDITIVE;
        o.flags = KF_COMPILE_CODEGEN_ONLY;
        o.table = T.data();
        o.table_len = (int32_t)T.size();
        kf_plan* p = nullptr;
        if (kf_compile(s, &o, &p) == KF_OK) {
            exercise_plan(p);
            kf_plan_destroy(p);
        }
        // per-kernel parameters, and too many of them
        kf_impl_params kp[3];
        std::memset(kp, 0, sizeof kp);
        kp[0].mat_k = 2; kp[0].mat_waves = 4; kp[0].mat_group = 2; kp[0].mat_rows = 64;
        kp[1].mat_sched = 1; kp[1].mat_waves = 16; kp[1].mat_group = 2;
        kf_compile_opts_init(&o);
        o.flags = KF_COMPILE_CODEGEN_ONLY;
        o.kernel_params = kp;
        o.kernel_params_len = 2;
        EXPECT(kf_compile(s, &o, &p) == KF_OK);
        if (p) {
            exercise_plan(p);
            kf_plan_destroy(p);
            p = nullptr;
        }
        o.kernel_params_len = 3;
        EXPECT(kf_compile(s, &o, &p) == KF_ERR_ARG);
        // every legal partition
        kf_planset* en = nullptr;
        EXPECT(kf_enumerate(s, 0, &en) == KF_OK);
        int32_t ne = 0, nc2 = 0;
        kf_planset_count(en, &ne);
        kf_script_num_calls(s, &nc2);
        std::vector<int32_t> part((size_t)nc2);
        for (int32_t i = 0; i < ne; ++i) {
            EXPECT(kf_planset_get(en, i, part.data(), nc2) == KF_OK);
            kf_compile_opts_init(&o);
            o.mode = KF_MODE_PARTITION;
            o.flags = KF_COMPILE_CODEGEN_ONLY;
            o.partition = part.data();
            o.partition_len = nc2;
            kf_plan* q = nullptr;
            EXPECT(kf_compile(s, &o, &q) == KF_OK);
            if (q) {
                exercise_plan(q);
                kf_plan_destroy(q);
            }
        }
        kf_planset_destroy(en);
        kf_script_destroy(s);
    }
    for (int64_t n : {5, 300, 4096}) {
        kf_script* s = mixed(n);
        kf_planset* ps = nullptr;
        EXPECT(kf_candidates(s, 16, nullptr, 0, &ps) == KF_OK);
        int32_t nc = 0;
        kf_planset_count(ps, &nc);
        for (int32_t i = 0; i < nc; ++i) {
            kf_plan* p = nullptr;
            if (kf_planset_compile(ps, i, KF_COMPILE_CODEGEN_ONLY, &p) != KF_OK) continue;
            exercise_plan(p);
            kf_plan_destroy(p);
        }
        kf_planset_destroy(ps);
        kf_script_destroy(s);
    }
    for (auto& sh : shapes) {
        kf_script* s = gemver(sh[0], sh[1], KF_COL_MAJOR);
        all_candidates(s, 0);
        kf_script_destroy(s);
    }
    for (int32_t dt : {KF_BF16, KF_FP8_E4M3})
        for (auto& sh : shapes) {
            kf_script* s = bicgk_q(sh[0], sh[1], dt);
            all_candidates(s, 0);
            kf_script_destroy(s);
        }
    for (uint64_t seed = 1; seed <= 40; ++seed) {
        kf_script* s = random_script(seed, seed % 3 == 0 ? 4099 : 96, 3 + (int)(seed % 7));
        all_candidates(s, 24);
        kf_script_destroy(s);
    }
    // recorder and compiler error paths
    {
        kf_script* s = nullptr;
        kf_script_create(&s);
        kf_value v = -1, A = -1, x = -1, y = -1, one = cst(s, 1.f);
        EXPECT(kf_vector(s, 0, &v) == KF_ERR_SHAPE);
        EXPECT(kf_matrix(s, 4, 9, 8, &v) == KF_ERR_SHAPE);
        A = mat(s, 7, 9);
        x = vec(s, 7);
        y = vec(s, 9);
        EXPECT(kf_gemv(s, one, A, x, KF_NONE, KF_NONE, &v) == KF_ERR_SHAPE);
        EXPECT(kf_gemtv(s, one, A, y, KF_NONE, KF_NONE, &v) == KF_ERR_SHAPE);
        EXPECT(kf_axpy(s, one, x, y, &v) == KF_ERR_SHAPE);
        EXPECT(kf_ger(s, one, A, y, x, &v) == KF_ERR_SHAPE);
        EXPECT(kf_gemv(s, one, 12345, y, KF_NONE, KF_NONE, &v) != KF_OK);
        kf_plan* p = nullptr;
        EXPECT(kf_compile(s, nullptr, &p) == KF_ERR_STATE);   // no calls yet
        kf_compile_opts o;
        kf_compile_opts_init(&o);
        o.mat_k = 3;
        EXPECT(kf_gemv(s, one, A, y, KF_NONE, KF_NONE, &v) == KF_OK);
        EXPECT(kf_compile(s, &o, &p) == KF_ERR_ARG);
        kf_script_destroy(s);
    }
    // batch layout (host only)
    {
        const int64_t cnt = 9;
        std::vector<int32_t> kind(cnt);
        std::vector<int64_t> n(cnt);
        std::vector<float> al(cnt, 1.5f), be(cnt, 0.5f);
        for (int64_t i = 0; i < cnt; ++i) {
            kind[i] = (int32_t)(i & 1);
            n[i] = 32 + 250 * i;
        }
        kf_batch* b = nullptr;
        EXPECT(kf_batch_create(cnt, kind.data(), n.data(), al.data(), be.data(), nullptr, &b) == KF_OK);
        if (b) {
            int64_t el = 0, off = 0, ld = 0, r = 0, w = 0;
            size_t wsb = 0;
            EXPECT(kf_batch_arena_elems(b, &el) == KF_OK && el > 0);
            EXPECT(kf_batch_workspace_bytes(b, &wsb) == KF_OK);
            for (int64_t i = 0; i < cnt; ++i) EXPECT(kf_batch_offset(b, i, 0, &off, &ld) == KF_OK && off + n[i] * ld <= el);
            EXPECT(kf_batch_bytes(b, &r, &w) == KF_OK && r > 0 && w > 0);
            size_t need = 0;
            EXPECT(kf_batch_describe(b, nullptr, 0, &need) == KF_OK);
            kf_batch_destroy(b);
        }
        n[0] = 5000;   // above the largest bucket
        EXPECT(kf_batch_create(cnt, kind.data(), n.data(), al.data(), be.data(), nullptr, &b) != KF_OK);
    }
    // damaged cost-model files are refused before any device work
    {
        const char* path = "host_sanitize_model.kfcm";
        const char* bodies[] = {"", "KFCM", "KFCMxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxxx"};
        for (const char* body : bodies) {
            FILE* fp = std::fopen(path, "wb");
            std::fwrite(body, 1, std::strlen(body), fp);
            std::fclose(fp);
            kf_costmodel* cm = nullptr;
            EXPECT(kf_costmodel_load(path, &cm) == KF_ERR_ARG);
        }
        kf_costmodel* cm = nullptr;
        EXPECT(kf_costmodel_load("/nonexistent/model.kfcm", &cm) == KF_ERR_ARG);
        // a model saved and loaded back, then the same file with one byte changed
        // (models hold device copies of their parameters: skipped with no device)
        const kf_status cs = kf_costmodel_create(16, 2, 3, &cm);
        EXPECT(cs == KF_OK || cs == KF_ERR_HIP);
        if (cs == KF_OK) {
            EXPECT(kf_costmodel_set_launch_us(cm, 2.5f) == KF_OK);
            EXPECT(kf_costmodel_save(cm, path) == KF_OK);
            int32_t h = 0, l = 0;
            int64_t np = 0;
            EXPECT(kf_costmodel_dims(cm, &h, &l, &np) == KF_OK && h == 16 && l == 2 && np > 0);
            kf_costmodel_destroy(cm);
            cm = nullptr;
            EXPECT(kf_costmodel_load(path, &cm) == KF_OK);
            if (cm) {
                std::vector<float> prm((size_t)np), mu(KF_FEATURE_DIM), sd(KF_FEATURE_DIM);
                double y[2];
                float lu = 0.f;
                EXPECT(kf_costmodel_get(cm, prm.data(), mu.data(), sd.data(), y, &lu) == KF_OK && lu == 2.5f);
                kf_costmodel_destroy(cm);
                cm = nullptr;
            }
            FILE* fp = std::fopen(path, "r+b");
            if (fp) {
                std::fseek(fp, 40, SEEK_SET);
                int c = std::fgetc(fp);
                std::fseek(fp, 40, SEEK_SET);
                std::fputc(c ^ 0x5a, fp);
                std::fclose(fp);
            }
            EXPECT(kf_costmodel_load(path, &cm) == KF_ERR_ARG);
        }
        std::remove(path);
    }
    // the MLP's host-side helpers
    {
        kf_mlp* m = nullptr;
        EXPECT(kf_mlp_create(KF_FEATURE_DIM, 128, 3, &m) == KF_OK);
        int64_t np = 0;
        EXPECT(kf_mlp_param_count(m, &np) == KF_OK && np > 0);
        std::vector<float> prm((size_t)np);
        EXPECT(kf_mlp_init_params(m, 7, prm.data()) == KF_OK);
        size_t wsb = 0;
        EXPECT(kf_mlp_workspace_bytes(m, 256, &wsb) == KF_OK && wsb > 0);
        kf_mlp_destroy(m);
    }
    std::printf("plans generated: %d\n", g_plans);
    std::printf(g_fail ? "host sanitize driver: FAILED\n" : "host sanitize driver: ok\n");
    return g_fail;
}
