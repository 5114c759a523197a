// batch.cpp -- batched uneven-size BiCGK / GEMVER: arena layout, work items,
// the persistent launch, the per-instance launch loop and graph capture.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "kf_batch_defs.h"
#include "kf_internal.h"

hipError_t kfb_launch(const kfb_inst* insts, const kfb_item* items, int nitems, int item0, int grid, int persistent,
                      float* arena, float* ws, unsigned* sync, unsigned spin_limit, hipStream_t st);
hipError_t kfb_resident_blocks(int* per_cu, int* cus);

using kf::set_error;

namespace {

const int kVecSlots[2] = {4, 8};  // BiCGK p r q s; GEMVER u1 v1 u2 v2 y z x w

int64_t align64(int64_t x) { return (x + 63) / 64 * 64; }  // 256-byte units of floats

// default rows per block: BiCGK keeps instances up to 512 whole and cuts
// larger ones into ~1 MiB blocks of A; GEMVER moves three times the bytes of
// A per row, so it is cut from n > 256 on.
const int kDefaultRows[2][KFB_BUCKETS] = {
    {64, 128, 256, 512, 256, 128},
    {64, 128, 256, 128, 128, 64},
};

struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
};

}  // namespace

struct kf_batch {
    std::vector<kfb_inst> insts;
    std::vector<kfb_item> queue;    // persistent order
    std::vector<kfb_item> by_inst;  // instance order (direct launches)
    std::vector<int32_t> first1, count1, first2, count2;  // ranges in by_inst
    int64_t arena_elems = 0, ws_floats = 0, sync_words = 0, nsplit = 0;
    int64_t bytes_read = 0, bytes_written = 0;
    int32_t rows[2][KFB_BUCKETS];
    int32_t tile[2][KFB_BUCKETS];   // entry of the tile menu per kind and bucket
    int32_t grid_req = 0;
    uint32_t spin_limit = 1u << 22;
    // bound state
    float* arena = nullptr;
    void* ws = nullptr;
    int grid = 0;
    Graph graphs[2];
    ~kf_batch() {
        for (Graph& g : graphs) {
            if (g.x) (void)hipGraphExecDestroy(g.x);
            if (g.g) (void)hipGraphDestroy(g.g);
        }
    }
    // Workspace layout, each part at a 256-byte boundary: the counters, the
    // column partials of split instances, then the instance table and the two
    // item tables (queue order and instance order), uploaded by kf_batch_bind.
    static size_t up256(size_t x) { return (x + 255) / 256 * 256; }
    size_t sync_bytes() const { return up256((size_t)sync_words * 4); }
    size_t part_bytes() const { return up256((size_t)ws_floats * 4); }
    size_t insts_bytes() const { return up256(insts.size() * sizeof(kfb_inst)); }
    size_t items_bytes() const { return up256(queue.size() * sizeof(kfb_item)); }
    size_t ws_bytes() const { return sync_bytes() + part_bytes() + insts_bytes() + 2 * items_bytes(); }
    unsigned* sync_ptr() const { return (unsigned*)ws; }
    float* part_ptr() const { return (float*)((char*)ws + sync_bytes()); }
    kfb_inst* insts_ptr() const { return (kfb_inst*)((char*)ws + sync_bytes() + part_bytes()); }
    kfb_item* queue_ptr() const { return (kfb_item*)((char*)insts_ptr() + insts_bytes()); }
    kfb_item* by_inst_ptr() const { return (kfb_item*)((char*)queue_ptr() + items_bytes()); }
};

extern "C" {

kf_status kf_batch_create(int64_t count, const int32_t* kind, const int64_t* n, const float* alpha,
                          const float* beta, const kf_batch_opts* opts, kf_batch** out) {
    if (!out || count < 0 || (count > 0 && (!kind || !n))) return set_error(KF_ERR_ARG, "bad argument");
    if (count > (1 << 24)) return set_error(KF_ERR_UNSUPPORTED, "at most 2^24 instances per batch");
    kf_batch* b = nullptr;
    try {
        b = new kf_batch();
    } catch (...) {
        return set_error(KF_ERR_NOMEM, "host allocation failed");
    }
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < KFB_BUCKETS; ++j) {
            b->rows[k][j] = kDefaultRows[k][j];
            b->tile[k][j] = 0;
        }
    if (opts) {
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < KFB_BUCKETS; ++j) {
                const int t = opts->tile[k][j];
                if (t < 0 || t >= kfb_tile_count(k, j)) {
                    delete b;
                    return set_error(KF_ERR_ARG, "tile is not on the menu of this kind and size bucket");
                }
                b->tile[k][j] = t;
                const int r = opts->rows[k][j];
                const int step = kfb_rows_per_step(k, j, t);
                if (r == 0) {
                    // the default rows per block, rounded up to the tile's rows per step
                    b->rows[k][j] = (kDefaultRows[k][j] + step - 1) / step * step;
                    continue;
                }
                if (r < 0 || r % step) {
                    delete b;
                    return set_error(KF_ERR_ARG, "rows per block must be a positive multiple of the tile's rows per step");
                }
                b->rows[k][j] = r;
            }
        if (opts->grid < 0) {
            delete b;
            return set_error(KF_ERR_ARG, "grid must be >= 0");
        }
        b->grid_req = opts->grid;
        if (opts->spin_limit) b->spin_limit = opts->spin_limit;
    }
    try {
        int64_t off = 0, wsf = 0;
        b->insts.resize(count);
        for (int64_t i = 0; i < count; ++i) {
            if (kind[i] != KF_BATCH_BICGK && kind[i] != KF_BATCH_GEMVER) {
                delete b;
                return set_error(KF_ERR_ARG, "instance kind must be KF_BATCH_BICGK or KF_BATCH_GEMVER");
            }
            if (n[i] < 1 || n[i] > KFB_MAX_N) {
                delete b;
                return set_error(KF_ERR_UNSUPPORTED, "instance size must be in [1, 2048]");
            }
            kfb_inst& I = b->insts[i];
            std::memset(&I, 0, sizeof(I));
            I.kind = kind[i];
            I.n = (int32_t)n[i];
            // rows start on 128-byte lines, so no line holds the end of one row and
            // the start of the next (stores of B and loads of A stay line-aligned)
            I.ld = (int32_t)((n[i] + 31) / 32 * 32);
            I.bucket = kfb_bucket(I.n);
            I.tile = b->tile[I.kind][I.bucket];
            I.rows = b->rows[I.kind][I.bucket];
            I.nblk = (I.n + I.rows - 1) / I.rows;
            if (I.nblk == 1) I.rows = I.n;
            I.alpha = alpha ? alpha[i] : 1.f;
            I.beta = beta ? beta[i] : 1.f;
            const int64_t mat = (int64_t)I.n * I.ld;
            I.a = off;
            off = align64(off + mat);
            if (I.kind == KF_BATCH_GEMVER) {
                I.b = off;
                off = align64(off + mat);
            } else {
                I.b = -1;
            }
            for (int v = 0; v < 8; ++v) {
                if (v < kVecSlots[I.kind]) {
                    I.v[v] = off;
                    off = align64(off + I.n);
                } else {
                    I.v[v] = -1;
                }
            }
            if (I.nblk > 1) {
                I.sync = (int32_t)b->nsplit++;
                I.ws = wsf;
                wsf = align64(wsf + (int64_t)I.nblk * I.ld);
            } else {
                I.sync = -1;
                I.ws = -1;
            }
            // algorithmic bytes of the fused plan of the instance
            const int64_t nn = I.n;
            if (I.kind == KF_BATCH_BICGK) {
                b->bytes_read += 4 * (nn * nn + 2 * nn);          // A, p, r
                b->bytes_written += 4 * 2 * nn;                  // q, s
            } else {
                b->bytes_read += 4 * (2 * nn * nn + 6 * nn + nn);  // A, six vectors | B, x
                b->bytes_written += 4 * (nn * nn + 2 * nn);       // B, x | w
            }
        }
        b->arena_elems = off;
        b->ws_floats = wsf;
        b->sync_words = KFB_SYNC_HEADER + KFB_SYNC_PER_INST * b->nsplit;

        // items in instance order
        b->first1.resize(count);
        b->count1.resize(count);
        b->first2.resize(count);
        b->count2.resize(count);
        for (int64_t i = 0; i < count; ++i) {
            const kfb_inst& I = b->insts[i];
            const int ph1 = I.kind == KF_BATCH_BICGK ? KFB_BICGK : KFB_GEMVER_K1;
            b->first1[i] = (int32_t)b->by_inst.size();
            b->count1[i] = I.nblk;
            for (int k = 0; k < I.nblk; ++k) b->by_inst.push_back({(int32_t)i, (ph1 << 24) | k});
            b->first2[i] = (int32_t)b->by_inst.size();
            b->count2[i] = (I.kind == KF_BATCH_GEMVER && I.nblk > 1) ? I.nblk : 0;
            for (int k = 0; k < b->count2[i]; ++k) b->by_inst.push_back({(int32_t)i, (KFB_GEMVER_K2 << 24) | k});
        }
        // persistent queue: phase-1 items, largest first (ties by instance and
        // block), then the K2 blocks in the order their instances started
        std::vector<std::pair<int64_t, int64_t>> key;  // (-cost, index in by_inst)
        for (int64_t i = 0; i < count; ++i) {
            const kfb_inst& I = b->insts[i];
            for (int k = 0; k < I.nblk; ++k) {
                const int64_t rows = std::min<int64_t>(I.rows, I.n - (int64_t)k * I.rows);
                int64_t cost = rows * I.ld;
                if (I.kind == KF_BATCH_GEMVER) cost *= (I.nblk == 1 ? 3 : 2);
                key.push_back({-cost, (int64_t)b->first1[i] + k});
            }
        }
        std::stable_sort(key.begin(), key.end());
        std::vector<int64_t> start(count, -1);
        for (size_t j = 0; j < key.size(); ++j) {
            const kfb_item it = b->by_inst[key[j].second];
            b->queue.push_back(it);
            if (start[it.inst] < 0) start[it.inst] = (int64_t)j;
        }
        std::vector<std::pair<int64_t, int64_t>> k2;
        for (int64_t i = 0; i < count; ++i)
            if (b->count2[i]) k2.push_back({start[i], i});
        std::sort(k2.begin(), k2.end());
        for (auto& e : k2)
            for (int k = 0; k < b->count2[e.second]; ++k) b->queue.push_back(b->by_inst[b->first2[e.second] + k]);
    } catch (const std::bad_alloc&) {
        delete b;
        return set_error(KF_ERR_NOMEM, "host allocation failed");
    }
    *out = b;
    return KF_OK;
}

void kf_batch_destroy(kf_batch* b) { delete b; }

kf_status kf_batch_arena_elems(const kf_batch* b, int64_t* elems) {
    if (!b || !elems) return set_error(KF_ERR_ARG, "null argument");
    *elems = b->arena_elems;
    return KF_OK;
}

kf_status kf_batch_workspace_bytes(const kf_batch* b, size_t* bytes) {
    if (!b || !bytes) return set_error(KF_ERR_ARG, "null argument");
    *bytes = b->ws_bytes();
    return KF_OK;
}

kf_status kf_batch_offset(const kf_batch* b, int64_t i, int32_t operand, int64_t* offset, int64_t* ld) {
    if (!b || !offset || i < 0 || i >= (int64_t)b->insts.size()) return set_error(KF_ERR_ARG, "bad argument");
    const kfb_inst& I = b->insts[i];
    int64_t off = -1;
    if (operand == 0) off = I.a;
    else if (operand == 1) off = I.b;
    else if (operand >= 2 && operand - 2 < kVecSlots[I.kind]) off = I.v[operand - 2];
    if (off < 0) return set_error(KF_ERR_ARG, "the instance has no such operand");
    *offset = off;
    if (ld) *ld = operand <= 1 ? I.ld : I.n;
    return KF_OK;
}

kf_status kf_batch_bytes(const kf_batch* b, int64_t* read, int64_t* written) {
    if (!b || !read || !written) return set_error(KF_ERR_ARG, "null argument");
    *read = b->bytes_read;
    *written = b->bytes_written;
    return KF_OK;
}

kf_status kf_batch_tile_info(int32_t kind, int32_t bucket, int32_t t, int32_t* count, int32_t* out) {
    if (kind < 0 || kind > 1 || bucket < 0 || bucket >= KFB_BUCKETS || t < 0 || !count)
        return set_error(KF_ERR_ARG, "bad kind, bucket or tile");
    const int c = kfb_tile_count(kind, bucket);
    if (t < c) {
        if (!out) return set_error(KF_ERR_ARG, "null argument");
        const kfb_tile& x = kfb_tile_menu[kind][bucket][t];
        out[0] = x.wide; out[1] = x.ltpr; out[2] = x.k; out[3] = x.lg;
        out[4] = kfb_rows_per_step(kind, bucket, t);
    }
    *count = c;
    return KF_OK;
}

kf_status kf_batch_describe(const kf_batch* b, char* buf, size_t len, size_t* needed) {
    if (!b) return set_error(KF_ERR_ARG, "null batch");
    int64_t per[2][KFB_BUCKETS] = {{0}}, split[2] = {0, 0}, ph1 = 0;
    for (const kfb_inst& I : b->insts) {
        per[I.kind][I.bucket]++;
        if (I.nblk > 1) split[I.kind]++;
        ph1 += I.nblk;
    }
    std::ostringstream o;
    o << "{\"instances\": " << b->insts.size() << ", \"items\": " << b->queue.size() << ", \"phase1_items\": " << ph1
      << ", \"split\": {\"bicgk\": " << split[0] << ", \"gemver\": " << split[1] << "}, \"buckets\": {";
    const char* names[2] = {"bicgk", "gemver"};
    for (int k = 0; k < 2; ++k) {
        o << (k ? ", " : "") << "\"" << names[k] << "\": [";
        for (int j = 0; j < KFB_BUCKETS; ++j) o << (j ? ", " : "") << per[k][j];
        o << "]";
    }
    o << "}, \"rows\": {";
    for (int k = 0; k < 2; ++k) {
        o << (k ? ", " : "") << "\"" << names[k] << "\": [";
        for (int j = 0; j < KFB_BUCKETS; ++j) o << (j ? ", " : "") << b->rows[k][j];
        o << "]";
    }
    o << "}, \"tiles\": {";
    for (int k = 0; k < 2; ++k) {
        o << (k ? ", " : "") << "\"" << names[k] << "\": [";
        for (int j = 0; j < KFB_BUCKETS; ++j) {
            const kfb_tile& t = kfb_tile_menu[k][j][b->tile[k][j]];
            o << (j ? ", " : "") << "\"" << (t.wide ? "wide" : "rows") << " tpr" << (t.wide ? 256 : (1 << t.ltpr))
              << " k" << (int)t.k << " g" << (1 << t.lg) << "\"";
        }
        o << "]";
    }
    o << "}, \"arena_elems\": " << b->arena_elems << ", \"workspace_bytes\": " << b->ws_bytes()
      << ", \"grid\": " << b->grid << ", \"bytes_read\": " << b->bytes_read << ", \"bytes_written\": "
      << b->bytes_written << "}";
    const std::string s = o.str();
    if (needed) *needed = s.size() + 1;
    if (buf && len) {
        std::strncpy(buf, s.c_str(), len - 1);
        buf[len - 1] = 0;
    }
    return KF_OK;
}

kf_status kf_batch_items(const kf_batch* b, int32_t which, int32_t* inst, int32_t* phase, int32_t* blk,
                         int64_t cap, int64_t* count) {
    if (!b || !count) return set_error(KF_ERR_ARG, "null argument");
    const std::vector<kfb_item>& v = which == 0 ? b->queue : b->by_inst;
    *count = (int64_t)v.size();
    for (int64_t j = 0; j < cap && j < (int64_t)v.size(); ++j) {
        if (inst) inst[j] = v[j].inst;
        if (phase) phase[j] = v[j].phase_blk >> 24;
        if (blk) blk[j] = v[j].phase_blk & 0xffffff;
    }
    return KF_OK;
}

kf_status kf_batch_bind(kf_batch* b, float* arena, void* workspace, void* stream) {
    if (!b || (!arena && b->arena_elems) || (!workspace && b->ws_bytes()))
        return set_error(KF_ERR_ARG, "null argument");
    if ((uintptr_t)arena % 256 || (uintptr_t)workspace % 256)
        return set_error(KF_ERR_ALIGN, "arena and workspace must be 256-byte aligned");
    const size_t ab = (size_t)b->arena_elems * 4;
    if (arena && workspace) {
        const char* x = (const char*)arena;
        const char* y = (const char*)workspace;
        if (x < y + b->ws_bytes() && y < x + ab) return set_error(KF_ERR_ALIAS, "workspace overlaps the arena");
    }
    hipStream_t st = (hipStream_t)stream;
    for (Graph& g : b->graphs) {
        if (g.x) (void)hipGraphExecDestroy(g.x);
        if (g.g) (void)hipGraphDestroy(g.g);
        g = Graph();
    }
    b->arena = arena;
    b->ws = workspace;
    if (workspace) {
        // clear the counters and upload the tables into the caller's workspace;
        // the host tables are read by the copies, so the stream is synchronised
        const size_t ni = b->insts.size() * sizeof(kfb_inst), nq = b->queue.size() * sizeof(kfb_item);
        if (hipMemsetAsync(workspace, 0, b->sync_bytes(), st) != hipSuccess ||
            (ni && hipMemcpyAsync(b->insts_ptr(), b->insts.data(), ni, hipMemcpyHostToDevice, st) != hipSuccess) ||
            (nq && hipMemcpyAsync(b->queue_ptr(), b->queue.data(), nq, hipMemcpyHostToDevice, st) != hipSuccess) ||
            (nq && hipMemcpyAsync(b->by_inst_ptr(), b->by_inst.data(), nq, hipMemcpyHostToDevice, st) != hipSuccess) ||
            hipStreamSynchronize(st) != hipSuccess) {
            b->ws = nullptr;
            return set_error(KF_ERR_HIP, "clearing the counters or uploading the batch tables failed");
        }
    }
    if (b->grid_req > 0) {
        b->grid = b->grid_req;
    } else {
        int per_cu = 0, cus = 0;
        if (kfb_resident_blocks(&per_cu, &cus) != hipSuccess || per_cu < 1 || cus < 1)
            return set_error(KF_ERR_HIP, "occupancy query failed");
        b->grid = per_cu * cus;
    }
    return KF_OK;
}

static kf_status batch_launch(kf_batch* b, int which, hipStream_t st) {
    if (!b->ws || (!b->arena && b->arena_elems)) return set_error(KF_ERR_UNBOUND, "kf_batch_bind first");
    if (b->insts.empty()) return KF_OK;
    const int nq = (int)b->queue.size();
    if (which == 0) {
        if (kfb_launch(b->insts_ptr(), b->queue_ptr(), nq, 0, b->grid, 1, b->arena, b->part_ptr(), b->sync_ptr(),
                       b->spin_limit, st) != hipSuccess)
            return set_error(KF_ERR_HIP, "persistent launch failed");
        return KF_OK;
    }
    for (size_t i = 0; i < b->insts.size(); ++i) {
        if (kfb_launch(b->insts_ptr(), b->by_inst_ptr(), nq, b->first1[i], b->count1[i], 0, b->arena, b->part_ptr(),
                       b->sync_ptr(), b->spin_limit, st) != hipSuccess ||
            kfb_launch(b->insts_ptr(), b->by_inst_ptr(), nq, b->first2[i], b->count2[i], 0, b->arena, b->part_ptr(),
                       b->sync_ptr(), b->spin_limit, st) != hipSuccess)
            return set_error(KF_ERR_HIP, "instance launch failed");
    }
    return KF_OK;
}

kf_status kf_batch_run(kf_batch* b, int32_t which, void* stream) {
    if (!b || which < 0 || which > 1) return set_error(KF_ERR_ARG, "bad argument");
    return batch_launch(b, which, (hipStream_t)stream);
}

kf_status kf_batch_capture(kf_batch* b, int32_t which, void* stream) {
    if (!b || which < 0 || which > 1 || !stream) return set_error(KF_ERR_ARG, "bad argument (capture needs a non-null stream)");
    Graph& g = b->graphs[which];
    if (g.x) (void)hipGraphExecDestroy(g.x);
    if (g.g) (void)hipGraphDestroy(g.g);
    g = Graph();
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return set_error(KF_ERR_HIP, "hipStreamBeginCapture failed");
    kf_status s = batch_launch(b, which, st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (s != KF_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess || !graph) return set_error(KF_ERR_HIP, "hipStreamEndCapture failed");
    g.g = graph;
    if (hipGraphInstantiate(&g.x, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        g = Graph();
        return set_error(KF_ERR_HIP, "hipGraphInstantiate failed");
    }
    return KF_OK;
}

kf_status kf_batch_graph_launch(kf_batch* b, int32_t which, void* stream) {
    if (!b || which < 0 || which > 1) return set_error(KF_ERR_ARG, "bad argument");
    if (!b->graphs[which].x) return set_error(KF_ERR_STATE, "kf_batch_capture first");
    if (hipGraphLaunch(b->graphs[which].x, (hipStream_t)stream) != hipSuccess)
        return set_error(KF_ERR_HIP, "hipGraphLaunch failed");
    return KF_OK;
}

kf_status kf_batch_time(kf_batch* b, int32_t which, int32_t graph, void* stream, int32_t warmup, int32_t reps,
                        float* median_us) {
    if (!b || !median_us || reps < 1 || warmup < 0 || which < 0 || which > 1) return set_error(KF_ERR_ARG, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    auto once = [&]() -> kf_status {
        return graph ? kf_batch_graph_launch(b, which, stream) : batch_launch(b, which, st);
    };
    for (int i = 0; i < warmup; ++i) {
        kf_status s = once();
        if (s != KF_OK) return s;
    }
    std::vector<hipEvent_t> ev(2 * reps, nullptr);
    kf_status out = KF_OK;
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) out = set_error(KF_ERR_HIP, "hipEventCreate");
    for (int i = 0; i < reps && out == KF_OK; ++i) {
        if (hipEventRecord(ev[2 * i], st) != hipSuccess) out = set_error(KF_ERR_HIP, "hipEventRecord");
        if (out == KF_OK) out = once();
        if (out == KF_OK && hipEventRecord(ev[2 * i + 1], st) != hipSuccess) out = set_error(KF_ERR_HIP, "hipEventRecord");
    }
    if (out == KF_OK && hipStreamSynchronize(st) != hipSuccess) out = set_error(KF_ERR_HIP, "hipStreamSynchronize");
    std::vector<float> t;
    for (int i = 0; i < reps && out == KF_OK; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) != hipSuccess) out = set_error(KF_ERR_HIP, "hipEventElapsedTime");
        t.push_back(ms * 1000.f);
    }
    for (auto& e : ev)
        if (e) (void)hipEventDestroy(e);
    if (out != KF_OK) return out;
    std::sort(t.begin(), t.end());
    *median_us = t[t.size() / 2];
    return KF_OK;
}

kf_status kf_batch_error(kf_batch* b, void* stream, uint32_t* bits) {
    if (!b || !bits) return set_error(KF_ERR_ARG, "null argument");
    if (!b->ws) return set_error(KF_ERR_UNBOUND, "kf_batch_bind first");
    hipStream_t st = (hipStream_t)stream;
    uint32_t v = 0;
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(&v, b->sync_ptr() + KFB_SYNC_ERROR, 4, hipMemcpyDeviceToHost) != hipSuccess)
        return set_error(KF_ERR_HIP, "reading the batch error word failed");
    // A dependent item that gave up its wait left its instance's counters
    // and x flag behind; with every run on the stream finished, clear all of
    // them (and the error word) so that the next run starts clean.
    if (v && (hipMemsetAsync(b->ws, 0, b->sync_bytes(), st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess))
        return set_error(KF_ERR_HIP, "clearing the batch counters failed");
    *bits = v;
    return KF_OK;
}

}  // extern "C"
