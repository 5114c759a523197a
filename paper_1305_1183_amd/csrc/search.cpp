// search.cpp -- plan ranking: the additive routine predictor, routine probes
// and the features of the learned cost model (Section 4.2).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <array>
#include <cstring>
#include <memory>
#include <numeric>
#include <set>

#include "kf_internal.h"

using namespace kf;

namespace {

// Environment classes of the routine table: 0 BLAS-1, 1 BLAS-2 column strips,
// 2 BLAS-2 row-resident (waves, group, rows as requested, 0 = default).
bool env_match(const kf_routine_entry& e, int cls, const MatParams& mp, const VecParams& vp) {
    if (e.cls != cls) return false;
    if (cls == 1) return e.env[0] == mp.k && e.env[1] == mp.waves && e.env[2] == mp.group && e.env[3] == mp.rows;
    if (cls == 2) return e.env[0] == mp.waves && e.env[1] == mp.group && e.env[2] == mp.rows;
    return e.env[0] == vp.unroll && e.env[1] == vp.threads && e.env[2] == vp.grid;
}

// The entry of `routine` in the environment whose extra LDS is nearest to the
// kernel's own LDS use (lds_bytes); ties go to the smaller amount.
const kf_routine_entry* find(const kf_routine_entry* t, int n, int cls, const MatParams& mp, const VecParams& vp,
                             int routine, size_t lds_bytes) {
    const kf_routine_entry* best = nullptr;
    double bd = 0;
    for (int i = 0; i < n; ++i) {
        if (t[i].routine != routine || !env_match(t[i], cls, mp, vp)) continue;
        const double d = std::fabs((double)t[i].lds_kb * 1024.0 - (double)lds_bytes);
        if (!best || d < bd || (d == bd && t[i].lds_kb < best->lds_kb)) { best = &t[i]; bd = d; }
    }
    return best;
}

}  // namespace

extern "C" {

kf_status kf_routine_time(int32_t routine, int64_t rows, int64_t cols, const kf_compile_opts* params,
                          int32_t extra_lds_kb, void* buf, size_t buf_bytes, void* stream, int32_t warmup,
                          int32_t reps, float* median_us) {
    if (!buf || !median_us || reps < 1 || warmup < 0) return set_error(KF_ERR_ARG, "bad argument");
    if (extra_lds_kb < 0 || extra_lds_kb > 96) return set_error(KF_ERR_ARG, "extra_lds_kb must be 0 .. 96");
    if (routine < 0 || routine >= KF_ROUTINE_FINISH) return set_error(KF_ERR_ARG, "routine has no probe");
    const bool mat = routine <= KF_ROUTINE_COMPUTE_GER;
    if (rows < 1 || (mat && (cols < 4 || cols % 4))) return set_error(KF_ERR_SHAPE, "probe shape");
    const size_t need = (mat ? (size_t)rows * cols * 4 : (size_t)rows * 4) + 65536;
    if (buf_bytes < need) return set_error(KF_ERR_WORKSPACE, "probe buffer too small");
    if ((uintptr_t)buf % 256) return set_error(KF_ERR_ALIGN, "probe buffer must be 256-byte aligned");
    MatParams mp;
    VecParams vp;
    if (params) {
        mp.k = params->mat_k; mp.waves = params->mat_waves; mp.group = params->mat_group; mp.rows = params->mat_rows;
        mp.sched = params->mat_sched;
        vp.unroll = params->vec_unroll; vp.threads = params->vec_threads; vp.grid = params->vec_grid;
    }
    if (mat && mp.sched == 1) {
        if (cols > 32768) return set_error(KF_ERR_UNSUPPORTED, "row-resident schedule needs cols <= 32768");
        const RowresGeom g = rowres_geometry(rows, cols, mp);
        if (g.G * g.WP > 64 || g.KP > 8 || g.R % g.G)
            return set_error(KF_ERR_ARG, "row-resident probe: bad waves, group or rows for this shape");
    } else if (mat) {
        MatParams q = default_mat_params(rows, cols, mp);
        if (q.rows % (q.waves * q.group)) return set_error(KF_ERR_ARG, "mat_rows must be a multiple of waves*group");
    }
    KernelCode kc;
    try {
        kc = generate_probe(routine, rows, cols, mp, vp, extra_lds_kb);
    } catch (...) {
        return set_error(KF_ERR_INTERNAL, "probe generation failed");
    }
    std::vector<void*> fns;
    kf_status st = load_kernel(kc, &fns);
    if (st != KF_OK) return st;
    const size_t data = mat ? (size_t)rows * cols * 4 : (size_t)rows * 4;
    void* src = buf;
    void* dst = buf;
    void* sink = (char*)buf + (data + 255) / 256 * 256;
    void* args[3] = {&src, &dst, &sink};
    hipStream_t s = (hipStream_t)stream;
    const Launch& l = kc.launches[0];
    auto launch = [&]() {
        return hipModuleLaunchKernel((hipFunction_t)fns[0], (unsigned)l.grid, 1, 1, (unsigned)l.block, 1, 1, 0, s,
                                     args, nullptr);
    };
    for (int i = 0; i < warmup; ++i)
        if (launch() != hipSuccess) return set_error(KF_ERR_HIP, "probe launch");
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return set_error(KF_ERR_HIP, "hipEventCreate");
    kf_status out = KF_OK;
    for (int i = 0; i < reps && out == KF_OK; ++i) {
        if (hipEventRecord(ev[2 * i], s) != hipSuccess || launch() != hipSuccess ||
            hipEventRecord(ev[2 * i + 1], s) != hipSuccess)
            out = set_error(KF_ERR_HIP, "probe launch");
    }
    std::vector<float> t;
    if (out == KF_OK && hipStreamSynchronize(s) != hipSuccess) out = set_error(KF_ERR_HIP, "sync");
    for (int i = 0; i < reps && out == KF_OK; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) out = set_error(KF_ERR_HIP, "elapsed");
        t.push_back(ms * 1000.f);
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (out != KF_OK) return out;
    std::sort(t.begin(), t.end());
    *median_us = t.size() % 2 ? t[t.size() / 2] : 0.5f * (t[t.size() / 2 - 1] + t[t.size() / 2]);
    return KF_OK;
}

}  // extern "C"

namespace {

// Added to the additive prediction of a kernel over the register budget: far
// above any real plan time, so such implementations are effectively pruned
constexpr double kOverBudgetUs = 1e9;

// Additive prediction of one kernel of a plan: max(t_t, t_c) plus the
// finishing launches (Section 4.2), with the kernel's own parameters.
kf_status predict_kernel_additive(const kf_plan* p, const PlanKernel& pk, const kf_routine_entry* table, int32_t n,
                                  double* us) {
    const KernelCode& kc = pk.code;
    const Space sp = call_space(p->s, kc.calls[0]);
    const bool mat = sp.mat;
    MatParams mp = mat ? default_mat_params(sp.a, sp.b, pk.mp) : MatParams();
    VecParams vp = mat ? VecParams() : default_vec_params(sp.a, pk.vp);
    if (!mat && pk.vp.grid > 0) vp.grid = pk.vp.grid;  // the environment is the requested point (grid is capped for short vectors)
    const bool rowres = mat && (pk.mp.sched == 1 || needs_rowres(p->s, kc.calls));
    MatParams rp = pk.mp;   // row-resident environment: the requested geometry (0 = default)
    if (rowres && rp.sched != 1) rp.waves = rp.group = rp.rows = 0;
    bool have_rowres = false;
    for (int i = 0; i < n && rowres && !have_rowres; ++i) have_rowres = table[i].cls == 2;
    const kf_routine_entry* first_mat = nullptr;
    for (int i = 0; i < n && rowres && !have_rowres && !first_mat; ++i)
        if (table[i].cls == 1) first_mat = &table[i];
    auto get = [&](int r) -> const kf_routine_entry* {
        if (rowres && have_rowres) return find(table, n, 2, rp, vp, r, kc.lds_bytes);
        if (rowres && first_mat) {
            // a table without row-resident probes: the routines of its first
            // BLAS-2 environment stand in
            MatParams e;
            e.k = first_mat->env[0]; e.waves = first_mat->env[1]; e.group = first_mat->env[2]; e.rows = first_mat->env[3];
            return find(table, n, 1, e, vp, r, kc.lds_bytes);
        }
        return find(table, n, mat ? 1 : 0, mp, vp, r, kc.lds_bytes);
    };
    double tt = 0, tc = 0;
    // transfers: every operand the kernel's launches move through HBM
    for (const Launch& l : kc.launches)
        for (const KArg& a : l.args) {
            if (a.value < 0) continue;
            const Value& x = p->s.values[a.value];
            double elems = x.kind == VK::Mat ? (double)x.rows * x.cols : x.kind == VK::Vec ? (double)x.n
                                                                          : x.kind == VK::DevScalar ? 1.0 : 0.0;
            if (elems == 0) continue;
            bool in = a.kind == ArgKind::MatIn || a.kind == ArgKind::VecIn || a.kind == ArgKind::DevScalarIn;
            bool outk = a.kind == ArgKind::MatOut || a.kind == ArgKind::VecOut || a.kind == ArgKind::DevScalarOut;
            if (!in && !outk) continue;
            int r;
            if (mat) r = in ? KF_ROUTINE_LOAD_MAT : KF_ROUTINE_STORE_MAT;  // vectors priced per element as matrix data
            else r = in ? KF_ROUTINE_LOAD_VEC : KF_ROUTINE_STORE_VEC;
            const kf_routine_entry* e = get(r);
            if (!e) return set_error(KF_ERR_UNSUPPORTED, "routine table has no transfer entry for this environment");
            tt += elems * e->us_per_unit;
        }
    for (int c : kc.calls) {
        int r = -1;
        switch (p->s.calls[c].op) {
            case Op::Scal: r = KF_ROUTINE_COMPUTE_SCAL; break;
            case Op::Axpy: r = KF_ROUTINE_COMPUTE_AXPY; break;
            case Op::Dot: r = KF_ROUTINE_COMPUTE_DOT; break;
            case Op::Gemv: r = KF_ROUTINE_COMPUTE_GEMV; break;
            case Op::Gemtv: r = KF_ROUTINE_COMPUTE_GEMTV; break;
            case Op::Ger: r = KF_ROUTINE_COMPUTE_GER; break;
        }
        const kf_routine_entry* e = get(r);
        if (!e) return set_error(KF_ERR_UNSUPPORTED, "routine table has no compute entry for this environment");
        tc += (mat ? (double)sp.a * sp.b : (double)sp.a) * e->us_per_unit;
    }
    double t = std::max(tt, tc);
    if (kc.launches.size() > 1) {
        const kf_routine_entry* e = get(KF_ROUTINE_FINISH);
        if (!e) return set_error(KF_ERR_UNSUPPORTED, "routine table has no FINISH entry for this environment");
        t += (double)(kc.launches.size() - 1) * e->us_per_unit;
    }
    // Section 4.2 prunes fusion implementations that need more on-chip memory
    // than another implementation of the same fusion. On gfx950 the on-chip
    // memory a row-resident kernel outgrows is its registers: an implementation
    // over the register budget ranks after every one within it (the routine
    // times, probed one routine at a time, cannot show its spills).
    if (kc.over_budget) t += kOverBudgetUs;
    *us = t;
    return KF_OK;
}

}  // namespace

extern "C" {

kf_status kf_predict_additive(const kf_plan* p, const kf_routine_entry* table, int32_t n, float* us) {
    if (!p || !table || !us || n < 1) return set_error(KF_ERR_ARG, "bad argument");
    double total = 0;
    for (const PlanKernel& pk : p->ks) {
        double t = 0;
        kf_status st = predict_kernel_additive(p, pk, table, n, &t);
        if (st != KF_OK) return st;
        total += t;
    }
    *us = (float)total;
    return KF_OK;
}

kf_status kf_plan_features(const kf_plan* p, float* out, int32_t rows, int32_t* nk) {
    if (!p || !nk) return set_error(KF_ERR_ARG, "null argument");
    *nk = (int32_t)p->ks.size();
    if (!out) return KF_OK;
    if (rows < *nk) return set_error(KF_ERR_ARG, "feature buffer has too few rows");
    for (size_t k = 0; k < p->ks.size(); ++k)
        kernel_features(p->s, p->ks[k].code, p->part, p->ks[k].mp, p->ks[k].vp, out + k * KF_FEATURE_DIM);
    return KF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// candidates
// ---------------------------------------------------------------------------
namespace {

kf_compile_opts cand_opts(const kf_planset* ps, int i) {
    kf_compile_opts o = ps->params[i];
    o.mode = KF_MODE_PARTITION;
    o.partition = ps->parts[i].data();
    o.partition_len = (int32_t)ps->parts[i].size();
    o.table = nullptr;
    o.table_len = 0;
    o.grid = nullptr;
    o.grid_len = 0;
    return o;
}

// Default parameter points: the library's shape-dependent defaults (all zero),
// the autotuner's best points for large shapes, and the row-resident schedule.
std::vector<kf_compile_opts> default_grid() {
    std::vector<kf_compile_opts> g;
    const int mat[][5] = {{0, 0, 0, 0, 0}, {1, 4, 4, 1024, 0}, {2, 8, 2, 1024, 0}, {1, 4, 4, 256, 0},
                          {2, 4, 4, 512, 0}, {1, 4, 2, 1024, 0}, {2, 4, 2, 2048, 0}, {0, 8, 2, 0, 1}};
    const int vec[][3] = {{0, 0, 0}, {4, 256, 2048}, {4, 256, 4096}, {2, 256, 1024}};
    for (auto& m : mat)
        for (auto& v : vec) {
            kf_compile_opts o;
            kf_compile_opts_init(&o);
            o.mat_k = m[0]; o.mat_waves = m[1]; o.mat_group = m[2]; o.mat_rows = m[3]; o.mat_sched = m[4];
            o.vec_unroll = v[0]; o.vec_threads = v[1]; o.vec_grid = v[2];
            g.push_back(o);
        }
    return g;
}

}  // namespace

extern "C" {

kf_status kf_candidates(const kf_script* s, int32_t max_partitions, const kf_compile_opts* grid, int32_t grid_len,
                        kf_planset** out) {
    if (!s || !out) return set_error(KF_ERR_ARG, "null argument");
    if (s->s.calls.empty()) return set_error(KF_ERR_STATE, "script has no calls");
    try {
        auto* ps = new kf_planset();
        std::unique_ptr<kf_planset> guard(ps);
        ps->s = s->s;
        ps->candidates = true;
        std::vector<kf_compile_opts> g = grid && grid_len > 0 ? std::vector<kf_compile_opts>(grid, grid + grid_len)
                                                              : default_grid();
        auto parts = enumerate_partitions(s->s, max_partitions > 0 ? max_partitions : 64);
        bool has_mat = false, has_vec = false;
        for (size_t c = 0; c < s->s.calls.size(); ++c) (call_space(s->s, (int)c).mat ? has_mat : has_vec) = true;
        std::set<std::string> seen;
        for (const auto& part : parts)
            for (const auto& go : g) {
                kf_compile_opts o = go;
                if (!has_mat) o.mat_k = o.mat_waves = o.mat_group = o.mat_rows = o.mat_sched = 0;
                if (!has_vec) o.vec_unroll = o.vec_threads = o.vec_grid = 0;
                o.mode = KF_MODE_PARTITION;
                o.partition = part.data();
                o.partition_len = (int32_t)part.size();
                o.table = nullptr; o.table_len = 0; o.grid = nullptr; o.grid_len = 0;
                o.kernel_params = nullptr; o.kernel_params_len = 0;   // a grid point is one point for all kernels
                o.model = nullptr; o.bind_values = nullptr; o.bind_ptrs = nullptr; o.bind_len = 0;
                o.flags = KF_COMPILE_CODEGEN_ONLY;
                kf_plan* p = nullptr;
                if (build_plan(s->s, part, o, &p) != KF_OK) continue;  // illegal point for this shape
                std::string sig;
                for (auto& k : p->ks) sig += k.code.name + ",";
                kf_plan_destroy(p);
                if (!seen.insert(sig).second) continue;
                o.flags = 0;
                ps->parts.push_back(part);
                ps->params.push_back(o);
            }
        *out = guard.release();
    } catch (const std::bad_alloc&) {
        return set_error(KF_ERR_NOMEM, "host allocation failed");
    }
    return KF_OK;
}

kf_status kf_planset_params(const kf_planset* ps, int32_t i, kf_compile_opts* out) {
    if (!ps || !out || !ps->candidates) return set_error(KF_ERR_ARG, "not a candidate set");
    if (i < 0 || i >= (int32_t)ps->parts.size()) return set_error(KF_ERR_ARG, "index out of range");
    *out = cand_opts(ps, i);
    return KF_OK;
}

kf_status kf_planset_compile(const kf_planset* ps, int32_t i, int32_t flags, kf_plan** out) {
    if (!ps || !out || !ps->candidates) return set_error(KF_ERR_ARG, "not a candidate set");
    if (i < 0 || i >= (int32_t)ps->parts.size()) return set_error(KF_ERR_ARG, "index out of range");
    kf_compile_opts o = cand_opts(ps, i);
    o.flags = flags;
    try {
        return build_plan(ps->s, ps->parts[i], o, out);
    } catch (const std::bad_alloc&) {
        return set_error(KF_ERR_NOMEM, "host allocation failed");
    }
}

kf_status kf_planset_precompile(const kf_planset* ps, const int32_t* idx, int32_t n) {
    if (!ps || !ps->candidates || (n > 0 && !idx)) return set_error(KF_ERR_ARG, "bad argument");
    std::vector<kf_plan*> plans;
    std::vector<const KernelCode*> ks;
    std::set<std::string> names;
    kf_status st = KF_OK;
    for (int j = 0; j < n && st == KF_OK; ++j) {
        kf_plan* p = nullptr;
        st = kf_planset_compile(ps, idx[j], KF_COMPILE_CODEGEN_ONLY, &p);
        if (st != KF_OK) break;
        plans.push_back(p);
        for (auto& k : p->ks)
            if (names.insert(k.code.name).second) ks.push_back(&k.code);
    }
    std::string log;
    if (st == KF_OK && !jit_precompile(ks, &log)) st = set_error(KF_ERR_COMPILE, log);
    for (kf_plan* p : plans) kf_plan_destroy(p);
    return st;
}

kf_status kf_planset_predict_additive(const kf_planset* ps, const kf_routine_entry* table, int32_t table_len,
                                      float* pred_us) {
    if (!ps || !ps->candidates || !pred_us) return set_error(KF_ERR_ARG, "bad argument");
    for (size_t i = 0; i < ps->parts.size(); ++i) {
        kf_plan* p = nullptr;
        kf_status st = kf_planset_compile(ps, (int32_t)i, KF_COMPILE_CODEGEN_ONLY, &p);
        if (st != KF_OK) return st;
        st = kf_predict_additive(p, table, table_len, &pred_us[i]);
        kf_plan_destroy(p);
        if (st != KF_OK) return st;
    }
    return KF_OK;
}

}  // extern "C"

// ---- combinations of kernel implementations ------------------------------------
// Candidates that share a partition generate the same kernels in the same order,
// each with the candidate's parameter point. Because plan costs add over kernels
// (the predictors are additive; measured kernels run one after another), the
// cheapest plan for a partition takes, for every kernel, the cheapest point.
namespace kf {
namespace {

struct Combination {
    int first = -1;             // a candidate of the chosen partition (its earliest)
    std::vector<int32_t> pick;  // candidate whose implementation each kernel takes
    double total = 0;
};

// cost[i][k]: cost of kernel k of candidate i; an empty row = not costed.
Combination best_combination(const kf_planset* ps, const std::vector<std::vector<double>>& cost) {
    Combination best;
    std::vector<char> done(ps->parts.size(), 0);
    for (size_t i = 0; i < ps->parts.size(); ++i) {
        if (done[i]) continue;
        // the group of candidates with this partition, in candidate order
        std::vector<int32_t> grp;
        for (size_t j = i; j < ps->parts.size(); ++j)
            if (!done[j] && ps->parts[j] == ps->parts[i]) {
                done[j] = 1;
                if (!cost[j].empty()) grp.push_back((int32_t)j);
            }
        if (grp.empty()) continue;
        const size_t nk = cost[grp[0]].size();
        Combination c;
        c.first = grp[0];
        c.pick.assign(nk, -1);
        for (size_t k = 0; k < nk; ++k) {
            for (int32_t j : grp) {
                if (cost[j].size() != nk) continue;
                // within 0.1% counts as equal (Table 4): keep the earlier candidate
                if (c.pick[k] < 0 || cost[j][k] < cost[c.pick[k]][k] * 0.999) c.pick[k] = j;
            }
            c.total += cost[c.pick[k]][k];
        }
        // partitions come fewest kernels first: a later one must be 0.1% cheaper
        if (best.first < 0 || c.total < best.total * 0.999) best = c;
    }
    return best;
}

kf_status compile_combination(const kf_planset* ps, const Combination& c, int32_t flags, kf_plan** out) {
    if (c.first < 0) return set_error(KF_ERR_UNSUPPORTED, "no candidate could be costed");
    kf_compile_opts o;
    kf_compile_opts_init(&o);
    o.mode = KF_MODE_PARTITION;
    o.flags = flags;
    o.partition = ps->parts[c.first].data();
    o.partition_len = (int32_t)ps->parts[c.first].size();
    std::vector<kf_impl_params> kp(c.pick.size());
    for (size_t k = 0; k < c.pick.size(); ++k) {
        const kf_compile_opts& g = ps->params[c.pick[k]];
        kf_impl_params& e = kp[k];
        e.mat_k = g.mat_k; e.mat_waves = g.mat_waves; e.mat_group = g.mat_group; e.mat_rows = g.mat_rows;
        e.mat_sched = g.mat_sched; e.mat_unit = g.mat_unit;
        e.vec_unroll = g.vec_unroll; e.vec_threads = g.vec_threads; e.vec_grid = g.vec_grid;
    }
    o.kernel_params = kp.data();
    o.kernel_params_len = (int32_t)kp.size();
    try {
        return build_plan(ps->s, ps->parts[c.first], o, out);
    } catch (const std::bad_alloc&) {
        return set_error(KF_ERR_NOMEM, "host allocation failed");
    }
}

}  // namespace
}  // namespace kf

kf_status compile_additive(const kf_script* s, const kf_compile_opts& o, kf_plan** out) {
    if (!o.table || o.table_len < 1) return set_error(KF_ERR_ARG, "KF_MODE_ADDITIVE needs a routine table");
    std::vector<kf_compile_opts> grid;
    if (o.grid && o.grid_len > 0) {
        grid.assign(o.grid, o.grid + o.grid_len);
    } else {
        // every (BLAS-2 environment, BLAS-1 environment) pair present in the table
        // (class first: 1 column strips, 2 row-resident)
        std::vector<std::array<int, 5>> me, ve;
        for (int i = 0; i < o.table_len; ++i) {
            const kf_routine_entry& t = o.table[i];
            std::array<int, 5> e = {t.cls, t.env[0], t.env[1], t.env[2], t.env[3]};
            auto& v = t.cls ? me : ve;
            if (std::find(v.begin(), v.end(), e) == v.end()) v.push_back(e);
        }
        if (me.empty()) me.push_back({1, 0, 0, 0, 0});
        if (ve.empty()) ve.push_back({0, 0, 0, 0, 0});
        for (auto& m : me)
            for (auto& v : ve) {
                kf_compile_opts g;
                kf_compile_opts_init(&g);
                if (m[0] == 2) {
                    g.mat_sched = 1; g.mat_waves = m[1]; g.mat_group = m[2]; g.mat_rows = m[3];
                } else {
                    g.mat_k = m[1]; g.mat_waves = m[2]; g.mat_group = m[3]; g.mat_rows = m[4];
                }
                g.vec_unroll = v[1]; g.vec_threads = v[2]; g.vec_grid = v[3];
                grid.push_back(g);
            }
    }
    kf_planset* ps = nullptr;
    kf_status st = kf_candidates(s, o.max_partitions, grid.data(), (int32_t)grid.size(), &ps);
    if (st != KF_OK) return st;
    std::unique_ptr<kf_planset> guard(ps);
    std::vector<std::vector<double>> cost(ps->parts.size());
    for (size_t i = 0; i < ps->parts.size(); ++i) {
        kf_plan* p = nullptr;
        if (kf_planset_compile(ps, (int32_t)i, KF_COMPILE_CODEGEN_ONLY, &p) != KF_OK) continue;
        std::vector<double> c;
        for (const PlanKernel& pk : p->ks) {
            double us = 0;
            if (predict_kernel_additive(p, pk, o.table, o.table_len, &us) != KF_OK) {
                c.clear();
                break;
            }
            c.push_back(us);
        }
        kf_plan_destroy(p);
        cost[i] = std::move(c);
    }
    kf::Combination best = kf::best_combination(ps, cost);
    if (best.first < 0) return set_error(KF_ERR_UNSUPPORTED, "no candidate could be predicted with this routine table");
    return kf::compile_combination(ps, best, o.flags, out);
}

// ---- learned and empirical ranking inside kf_compile -------------------------
namespace kf {

kf_status costmodel_plan_us(kf_costmodel* cm, const std::vector<float>& feats, const std::vector<size_t>& start,
                            hipStream_t st, std::vector<double>* us);

namespace {

// Times candidates of a planset kernel by kernel with the caller's buffers and
// the caller's workspace (opts.workspace).
struct Timer {
    const kf_planset* ps;
    const kf_compile_opts& o;
    int too_big = 0;   // candidates whose workspace did not fit
    Timer(const kf_planset* p, const kf_compile_opts& opts) : ps(p), o(opts) {}
    kf_status time_kernels(int32_t i, std::vector<double>* us) {
        kf_plan* p = nullptr;
        kf_status s = kf_planset_compile(ps, i, 0, &p);
        if (s != KF_OK) return s;
        std::unique_ptr<kf_plan, void (*)(kf_plan*)> guard(p, kf_plan_destroy);
        for (int b = 0; b < o.bind_len; ++b) {
            s = kf_bind(p, o.bind_values[b], o.bind_ptrs[b]);
            if (s != KF_OK) return s;
        }
        size_t need = 0;
        kf_plan_workspace_bytes(p, &need);
        if (need > o.workspace_bytes || (need && !o.workspace)) {
            ++too_big;
            return set_error(KF_ERR_WORKSPACE, "candidate workspace larger than opts.workspace_bytes");
        }
        if (need) {
            s = kf_bind_workspace(p, o.workspace, o.workspace_bytes);
            if (s != KF_OK) return s;
        }
        std::vector<float> t(p->ks.size());
        s = kf_time_plan_kernels(p, o.stream, 2, 5, t.data());
        if (s != KF_OK) return s;
        us->assign(t.begin(), t.end());
        return KF_OK;
    }
};

kf_status candidates_for(const kf_script* s, const kf_compile_opts& o, kf_planset** ps) {
    return kf_candidates(s, o.max_partitions, o.grid_len > 0 ? o.grid : nullptr, o.grid_len > 0 ? o.grid_len : 0, ps);
}

// Times the candidates of `order` kernel by kernel and returns the cheapest
// combination of the measured implementations.
kf_status measured_combination(const kf_planset* ps, const kf_compile_opts& o, const std::vector<int32_t>& order,
                               Combination* best) {
    if (!o.bind_values || !o.bind_ptrs || o.bind_len < 1)
        return set_error(KF_ERR_UNBOUND, "timing candidates needs the buffers of opts.bind_values / bind_ptrs");
    if (o.time_budget_ms < 0) return set_error(KF_ERR_ARG, "time_budget_ms must be >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    kf_planset_precompile(ps, order.data(), (int32_t)order.size());
    Timer t(ps, o);
    std::vector<std::vector<double>> cost(ps->parts.size());
    bool any = false;
    for (int32_t i : order) {
        if (any && o.time_budget_ms > 0 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(o.time_budget_ms))
            break;
        std::vector<double> us;
        kf_status s = t.time_kernels(i, &us);
        if (s == KF_ERR_HIP || s == KF_ERR_UNBOUND || s == KF_ERR_ALIGN || s == KF_ERR_ALIAS) return s;
        if (s != KF_OK) continue;
        cost[i] = std::move(us);
        any = true;
    }
    *best = best_combination(ps, cost);
    if (best->first < 0) {
        if (t.too_big > 0 && !any)
            return set_error(KF_ERR_WORKSPACE, "no candidate fits opts.workspace_bytes (see kf_compile_workspace_bytes)");
        return set_error(KF_ERR_UNSUPPORTED, "no candidate could be timed");
    }
    return KF_OK;
}

}  // namespace

kf_status compile_learned(const kf_script* s, const kf_compile_opts& o, kf_plan** out) {
    if (!o.model) return set_error(KF_ERR_ARG, "KF_MODE_LEARNED needs opts.model");
    kf_planset* ps = nullptr;
    kf_status st = candidates_for(s, o, &ps);
    if (st != KF_OK) return st;
    std::unique_ptr<kf_planset> guard(ps);
    std::vector<float> feats;
    std::vector<size_t> row_of(ps->parts.size(), SIZE_MAX), nk_of(ps->parts.size(), 0);
    for (size_t i = 0; i < ps->parts.size(); ++i) {
        kf_plan* p = nullptr;
        if (kf_planset_compile(ps, (int32_t)i, KF_COMPILE_CODEGEN_ONLY, &p) != KF_OK) continue;
        int32_t nk = 0;
        kf_plan_features(p, nullptr, 0, &nk);
        const size_t at = feats.size();
        feats.resize(at + (size_t)nk * KF_FEATURE_DIM);
        kf_plan_features(p, feats.data() + at, nk, &nk);
        kf_plan_destroy(p);
        row_of[i] = at / KF_FEATURE_DIM;
        nk_of[i] = (size_t)nk;
    }
    const size_t rows = feats.size() / KF_FEATURE_DIM;
    if (rows == 0) return set_error(KF_ERR_UNSUPPORTED, "no candidate plan");
    // one prediction per kernel row (its launch term included)
    std::vector<size_t> start(rows + 1);
    std::iota(start.begin(), start.end(), 0);
    std::vector<double> kus;
    st = costmodel_plan_us(o.model, feats, start, (hipStream_t)o.stream, &kus);
    if (st != KF_OK) return st;
    std::vector<std::vector<double>> cost(ps->parts.size());
    std::vector<int32_t> ok;
    std::vector<double> plan_us;
    for (size_t i = 0; i < ps->parts.size(); ++i) {
        if (row_of[i] == SIZE_MAX) continue;
        cost[i].assign(kus.begin() + row_of[i], kus.begin() + row_of[i] + nk_of[i]);
        ok.push_back((int32_t)i);
        plan_us.push_back(std::accumulate(cost[i].begin(), cost[i].end(), 0.0));
    }
    Combination best = best_combination(ps, cost);
    if (o.top_k > 1) {
        // time the top_k candidates by predicted plan time (within 0.1%: the
        // earlier, fewer kernels, first) and the candidates of the predicted
        // combination, kernel by kernel; combine the measured implementations
        std::vector<size_t> order(ok.size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return plan_us[a] < plan_us[b] * 0.999; });
        std::vector<int32_t> timed;
        for (size_t j = 0; j < order.size() && (int)j < o.top_k; ++j) timed.push_back(ok[order[j]]);
        for (int32_t i : best.pick)
            if (std::find(timed.begin(), timed.end(), i) == timed.end()) timed.push_back(i);
        st = measured_combination(ps, o, timed, &best);
        if (st != KF_OK) return st;
    }
    return compile_combination(ps, best, o.flags, out);
}

kf_status timed_workspace_bytes(const kf_script* s, const kf_compile_opts& o, size_t* bytes) {
    kf_planset* ps = nullptr;
    kf_status st = candidates_for(s, o, &ps);
    if (st != KF_OK) return st;
    std::unique_ptr<kf_planset> guard(ps);
    size_t most = 0;
    for (size_t i = 0; i < ps->parts.size(); ++i) {
        kf_plan* p = nullptr;
        if (kf_planset_compile(ps, (int32_t)i, KF_COMPILE_CODEGEN_ONLY, &p) != KF_OK) continue;
        size_t need = 0;
        kf_plan_workspace_bytes(p, &need);
        kf_plan_destroy(p);
        most = std::max(most, need);
    }
    *bytes = most;
    return KF_OK;
}

kf_status compile_exhaustive(const kf_script* s, const kf_compile_opts& o, kf_plan** out) {
    kf_planset* ps = nullptr;
    kf_status st = candidates_for(s, o, &ps);
    if (st != KF_OK) return st;
    std::unique_ptr<kf_planset> guard(ps);
    std::vector<int32_t> all(ps->parts.size());
    std::iota(all.begin(), all.end(), 0);
    Combination best;
    st = measured_combination(ps, o, all, &best);
    if (st != KF_OK) return st;
    return compile_combination(ps, best, o.flags, out);
}

}  // namespace kf
