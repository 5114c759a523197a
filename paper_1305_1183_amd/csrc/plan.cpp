// plan.cpp -- data-dependency graph, fusion legality and plan enumeration.
//
// Section 4.2: the script's calls form a data-dependency graph; a *fusion* is
// a subgraph whose calls can share one kernel without changing the script's
// meaning; a plan (a "combination") covers every call with fusions and single
// calls. The legality rules follow Section 3.2:
//   R1  a kernel's call set is convex in the graph (no path leaves and
//       re-enters it), and the kernels of a plan form an acyclic graph;
//   R2  all calls of a kernel iterate over the same space -- calls of
//       different nesting depth (BLAS-1 vs BLAS-2) are never fused;
//   R3  a reduction result needs a global barrier, so it is not consumed in
//       the kernel that computes it (Section 3.2.2) -- except, as this
//       library's extension, as the additive y0 term of a reduction of the
//       same kind, which the last workgroup applies after its own barrier
//       (the "last running block" of Section 3.2.2);
//   R4  fusions that share no data save no transfers and are pruned.
#include <algorithm>
#include <functional>
#include <numeric>
#include <sstream>

#include "kf_internal.h"

namespace kf {

const char* op_name(Op op) {
    switch (op) {
        case Op::Scal: return "scal";
        case Op::Axpy: return "axpy";
        case Op::Dot: return "dot";
        case Op::Gemv: return "gemv";
        case Op::Gemtv: return "gemtv";
        case Op::Ger: return "ger";
    }
    return "?";
}

bool is_reduction(Op op) { return op == Op::Dot || op == Op::Gemv || op == Op::Gemtv; }

Space call_space(const Script& s, int c) {
    const Call& k = s.calls[c];
    Space sp;
    if (k.op == Op::Gemv || k.op == Op::Gemtv || k.op == Op::Ger) {
        const Value& A = s.values[k.in[0]];
        sp.mat = true;
        sp.a = A.rows;
        sp.b = A.cols;
    } else {
        sp.mat = false;
        sp.a = s.values[k.in[0]].n;
        sp.b = 0;
    }
    return sp;
}

// Data values (vectors, matrices) a call touches, inputs and output.
static std::vector<int> call_data(const Script& s, int ci) {
    std::vector<int> v;
    const Call& c = s.calls[ci];
    for (int i = 0; i < 3; ++i)
        if (c.in[i] >= 0) {
            VK k = s.values[c.in[i]].kind;
            if (k == VK::Vec || k == VK::Mat) v.push_back(c.in[i]);
        }
    VK k = s.values[c.out].kind;
    if (k == VK::Vec || k == VK::Mat) v.push_back(c.out);
    return v;
}

// Is the use of value `v` by call `d` the additive y0 term only?
static bool used_only_as_y0(const Call& d, int v) {
    if (d.alpha == v || d.beta == v) return false;
    if (d.in[0] == v || d.in[1] == v) return false;
    return d.in[2] == v;
}

std::string block_illegal_reason(const Script& s, const std::vector<int>& calls) {
    if (calls.empty()) return "empty";
    std::vector<char> in(s.calls.size(), 0);
    for (int c : calls) in[c] = 1;
    // R2: one iteration space.
    Space sp0 = call_space(s, calls[0]);
    for (int c : calls)
        if (!(call_space(s, c) == sp0)) return "R2: calls iterate over different spaces";
    // R3 (+ the same-kind y0 extension).
    for (int c : calls) {
        const Call& k = s.calls[c];
        if (!is_reduction(k.op)) continue;
        for (int d : s.values[k.out].consumers) {
            if (!in[d]) continue;
            const Call& kd = s.calls[d];
            bool ok = (k.op == Op::Gemv || k.op == Op::Gemtv) && kd.op == k.op &&
                      used_only_as_y0(kd, k.out);
            // R3'': a row dot may feed the row-indexed x of a gemtv when the kernel
            // keeps whole rows in one workgroup (row-resident schedule, cols <= 32768)
            if (!ok && k.op == Op::Gemv && kd.op == Op::Gemtv && kd.in[1] == k.out && kd.in[0] != k.out &&
                kd.in[2] != k.out && kd.alpha != k.out && kd.beta != k.out && call_space(s, c).b <= 32768 &&
                s.values[k.in[0]].dtype == KF_F32 && s.values[kd.in[0]].dtype == KF_F32)
                ok = true;
            if (!ok)
                return std::string("R3: result of ") + op_name(k.op) +
                       " consumed inside the kernel that reduces it";
        }
    }
    // R1: convexity -- no path from the set through an outside call back in.
    {
        std::vector<char> seen(s.calls.size(), 0);
        std::vector<int> stack;
        for (int c : calls)
            for (int d : s.values[s.calls[c].out].consumers)
                if (!in[d] && !seen[d]) { seen[d] = 1; stack.push_back(d); }
        while (!stack.empty()) {
            int d = stack.back();
            stack.pop_back();
            for (int e : s.values[s.calls[d].out].consumers) {
                if (in[e]) return "R1: a path leaves the kernel and re-enters it";
                if (!seen[e]) { seen[e] = 1; stack.push_back(e); }
            }
        }
    }
    // R4: connected through shared vectors or matrices.
    if (calls.size() > 1) {
        std::vector<int> comp(calls.size());
        std::iota(comp.begin(), comp.end(), 0);
        std::function<int(int)> find = [&](int x) { return comp[x] == x ? x : comp[x] = find(comp[x]); };
        for (size_t i = 0; i < calls.size(); ++i) {
            auto di = call_data(s, calls[i]);
            for (size_t j = i + 1; j < calls.size(); ++j) {
                auto dj = call_data(s, calls[j]);
                bool share = false;
                for (int a : di)
                    for (int b : dj)
                        if (a == b) share = true;
                if (share) comp[find((int)i)] = find((int)j);
            }
        }
        int root = find(0);
        for (size_t i = 1; i < calls.size(); ++i)
            if (find((int)i) != root) return "R4: the calls share no vector or matrix";
    }
    return "";
}

bool partition_acyclic(const Script& s, const std::vector<int>& part, int nk) {
    std::vector<std::set<int>> succ(nk);
    for (size_t c = 0; c < s.calls.size(); ++c)
        for (int d : s.values[s.calls[c].out].consumers)
            if (part[d] != part[c]) succ[part[c]].insert(part[d]);
    std::vector<int> indeg(nk, 0);
    for (int k = 0; k < nk; ++k)
        for (int t : succ[k]) indeg[t]++;
    std::vector<int> q;
    for (int k = 0; k < nk; ++k)
        if (!indeg[k]) q.push_back(k);
    int seen = 0;
    while (!q.empty()) {
        int k = q.back();
        q.pop_back();
        ++seen;
        for (int t : succ[k])
            if (--indeg[t] == 0) q.push_back(t);
    }
    return seen == nk;
}

static std::vector<int> canonical(const std::vector<int>& part) {
    std::map<int, int> ren;
    std::vector<int> out(part.size());
    for (size_t i = 0; i < part.size(); ++i) {
        auto it = ren.find(part[i]);
        if (it == ren.end()) it = ren.emplace(part[i], (int)ren.size()).first;
        out[i] = it->second;
    }
    return out;
}

std::vector<std::vector<int>> enumerate_partitions(const Script& s, int max_plans) {
    const int n = (int)s.calls.size();
    std::vector<std::vector<int>> result;
    if (n == 0) return result;
    // Candidate blocks: legal subsets of each iteration-space group.
    std::map<Space, std::vector<int>> groups;
    for (int c = 0; c < n; ++c) groups[call_space(s, c)].push_back(c);
    std::vector<std::vector<std::vector<int>>> blocks_with(n);  // blocks whose min call is c
    for (auto& g : groups) {
        const auto& mem = g.second;
        const int gsz = (int)mem.size();
        if (gsz > 20) {
            // Too many subsets to list: only singletons.
            for (int c : mem) blocks_with[c].push_back({c});
            continue;
        }
        for (uint32_t mask = 1; mask < (1u << gsz); ++mask) {
            std::vector<int> b;
            for (int i = 0; i < gsz; ++i)
                if (mask & (1u << i)) b.push_back(mem[i]);
            if (b.size() == 1 || block_illegal_reason(s, b).empty()) blocks_with[b[0]].push_back(b);
        }
    }
    // Exact covers by blocks, then the acyclicity check of the plan.
    const size_t hard_cap = 200000;
    std::vector<int> part(n, -1);
    int nk = 0;
    std::function<void(int)> rec = [&](int first) {
        if (result.size() >= hard_cap) return;
        while (first < n && part[first] >= 0) ++first;
        if (first == n) {
            if (partition_acyclic(s, part, nk)) result.push_back(canonical(part));
            return;
        }
        for (const auto& b : blocks_with[first]) {
            bool free_ = true;
            for (int c : b)
                if (part[c] >= 0) { free_ = false; break; }
            if (!free_) continue;
            for (int c : b) part[c] = nk;
            ++nk;
            rec(first + 1);
            --nk;
            for (int c : b) part[c] = -1;
        }
    };
    rec(0);
    auto nkern = [](const std::vector<int>& p) { return *std::max_element(p.begin(), p.end()) + 1; };
    std::stable_sort(result.begin(), result.end(), [&](const std::vector<int>& a, const std::vector<int>& b) {
        int ka = nkern(a), kb = nkern(b);
        if (ka != kb) return ka < kb;
        return a < b;
    });
    if (max_plans > 0 && (int)result.size() > max_plans) result.resize(max_plans);
    return result;
}

std::vector<int> fused_partition(const Script& s) {
    auto all = enumerate_partitions(s, 1);
    if (all.empty()) return unfused_partition(s);
    return all[0];
}

std::vector<int> unfused_partition(const Script& s) {
    std::vector<int> p(s.calls.size());
    std::iota(p.begin(), p.end(), 0);
    return p;
}

std::vector<std::vector<int>> kernels_in_order(const Script& s, const std::vector<int>& part) {
    int nk = part.empty() ? 0 : *std::max_element(part.begin(), part.end()) + 1;
    std::vector<std::vector<int>> members(nk);
    for (size_t c = 0; c < part.size(); ++c) members[part[c]].push_back((int)c);
    std::vector<std::set<int>> succ(nk);
    std::vector<int> indeg(nk, 0);
    for (size_t c = 0; c < s.calls.size(); ++c)
        for (int d : s.values[s.calls[c].out].consumers)
            if (part[d] != part[c] && succ[part[c]].insert(part[d]).second) indeg[part[d]]++;
    std::vector<std::vector<int>> order;
    std::set<std::pair<int, int>> ready;  // (first call, kernel)
    for (int k = 0; k < nk; ++k)
        if (!indeg[k]) ready.insert({members[k][0], k});
    while (!ready.empty()) {
        int k = ready.begin()->second;
        ready.erase(ready.begin());
        order.push_back(members[k]);
        for (int t : succ[k])
            if (--indeg[t] == 0) ready.insert({members[t][0], t});
    }
    return order;
}

int dtype_size(int dtype) { return dtype == KF_BF16 ? 2 : dtype == KF_FP8_E4M3 ? 1 : 4; }

int kernel_unit_elems(const Script& s, const std::vector<int>& calls, int req) {
    int es = 4;
    bool ger_q = false;
    for (int c : calls) {
        const Value& A = s.values[s.calls[c].in[0]];
        if (A.kind == VK::Mat) es = std::min(es, dtype_size(A.dtype));
        if (A.kind == VK::Mat && A.dtype != KF_F32 && s.calls[c].op == Op::Ger) ger_q = true;
    }
    // req: 4 = narrow units (four elements per lane and load), 16 = one
    // 16-byte load per lane; 0 = automatic. Automatically, a kernel that
    // expands a quantised matrix into an FP32 one (ger) takes narrow units so
    // that its FP32 stores stay 16 bytes per lane and contiguous across the
    // wave; other kernels take 16-byte loads.
    if (es == 4 || req == 4) return 4;
    if (req == 16) return 16 / es;
    if (ger_q) return 4;
    return 16 / es;
}

bool kernel_has_quantized(const Script& s, const std::vector<int>& calls) {
    for (int c : calls) {
        const Value& A = s.values[s.calls[c].in[0]];
        if (A.kind == VK::Mat && A.dtype != KF_F32) return true;
    }
    return false;
}

MatParams default_mat_params(int64_t rows, int64_t cols, const MatParams& req, int e_per_unit) {
    MatParams p = req;
    if (p.k <= 0) p.k = 1;
    if (p.waves <= 0) p.waves = 4;
    if (p.group <= 0) p.group = 4;
    const int unit = p.waves * p.group;
    if (p.rows <= 0) {
        const int64_t C = 64LL * e_per_unit * p.k;
        const int64_t S = (cols + C - 1) / C;
        // Aim for about 2048 workgroups (8 per CU) with at most 512 rows each.
        int64_t want_nb = (2048 + S - 1) / S;
        int64_t r = (rows + want_nb - 1) / want_nb;
        r = ((r + unit - 1) / unit) * unit;
        if (r < unit) r = unit;
        if (r > 512) r = (512 / unit) * unit;
        if (r < unit) r = unit;
        p.rows = (int)r;
    }
    return p;
}

VecParams default_vec_params(int64_t n, const VecParams& req) {
    VecParams p = req;
    if (p.unroll <= 0) p.unroll = 4;
    if (p.threads <= 0) p.threads = 256;
    int64_t n4 = n / 4;
    int64_t need = (n4 + (int64_t)p.threads * p.unroll - 1) / ((int64_t)p.threads * p.unroll);
    if (need < 1) need = 1;
    if (p.grid <= 0) p.grid = 2048;
    if (need < p.grid) p.grid = (int)need;
    return p;
}

}  // namespace kf
