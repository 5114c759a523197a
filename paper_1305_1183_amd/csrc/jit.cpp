// jit.cpp -- run-time compilation of generated kernels with hipRTC for gfx950.
//
// The paper's compiler emits CUDA source and hands it to the vendor compiler
// (Section 4.3); here every generated kernel is compiled in-process by hipRTC
// into a gfx950 code object: the building blocks plus the launches of one plan
// kernel, or of all the kernels of a plan not compiled yet. Code objects are
// cached in memory and, when a cache directory is set (kf_jit_set_cache_dir,
// else KF_CACHE_DIR), on disk under a hash of the unit's text and options, so
// that separate processes can compile candidate plans in parallel and the
// process that times them only loads the results.
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <sys/stat.h>
#include <unistd.h>

#include "kf_internal.h"

namespace kf {

static const char kBlocksText[] =
#include "kf_blocks_embed.inc"
    ;

static const char* kOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};

const std::string& blocks_source() {
    static const std::string s(kBlocksText);
    return s;
}

static uint64_t fnv1a64(const std::string& s, uint64_t h = 1469598103934665603ULL) {
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ULL;
    }
    return h;
}

// KF_JIT_EXTRA_SOURCE (debugging and tests): text appended to every generated
// translation unit, e.g. instrumentation, or an #error to exercise the
// compile-failure path. It is part of the text, so it is part of the cache key.
static std::string unit_text(const KernelCode& k) {
    std::string t = blocks_source() + "\n" + k.source;
    if (const char* extra = std::getenv("KF_JIT_EXTRA_SOURCE")) t += std::string("\n") + extra + "\n";
    return t;
}

// The disk cache directory: the one set through kf_jit_set_cache_dir, else
// KF_CACHE_DIR from the environment, else none.
static std::mutex g_dir_mu;
static bool g_dir_set = false;
static std::string g_dir;

static std::string cache_dir() {
    {
        std::lock_guard<std::mutex> lock(g_dir_mu);
        if (g_dir_set) return g_dir;
    }
    const char* dir = std::getenv("KF_CACHE_DIR");
    return dir ? std::string(dir) : std::string();
}

void jit_set_cache_dir(const char* dir, bool use_env) {
    std::lock_guard<std::mutex> lock(g_dir_mu);
    g_dir_set = !use_env;
    g_dir = dir ? dir : "";
}

static std::string cache_path(const std::string& text) {
    const std::string dir = cache_dir();
    if (dir.empty()) return "";
    std::string key = text;
    for (const char* o : kOpts) key += std::string("\n") + o;
    char name[64];
    std::snprintf(name, sizeof name, "/kf_%016llx.co", (unsigned long long)fnv1a64(key));
    return std::string(dir) + name;
}

// Cached code objects are stored as "KFCO", the FNV-1a 64 hash of the code
// object (8 bytes, host order) and the code object; a file that does not
// check out (truncated, overwritten) is ignored and rebuilt.
static bool read_file(const std::string& path, std::string* out) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::ostringstream ss;
    ss << f.rdbuf();
    const std::string d = ss.str();
    if (d.size() <= 12 || d.compare(0, 4, "KFCO") != 0) return false;
    uint64_t h = 0;
    std::memcpy(&h, d.data() + 4, 8);
    std::string co = d.substr(12);
    if (fnv1a64(co) != h) return false;
    *out = std::move(co);
    return true;
}

static std::string with_header(const std::string& co) {
    const uint64_t h = fnv1a64(co);
    std::string d = "KFCO";
    d.append(reinterpret_cast<const char*>(&h), 8);
    return d + co;
}

static void write_file_atomic(const std::string& path, const std::string& data) {
    std::string tmp = path + ".tmp" + std::to_string((long long)std::rand()) + std::to_string((long long)(uintptr_t)&data);
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f.write(data.data(), (std::streamsize)data.size());
    }
    std::rename(tmp.c_str(), path.c_str());
}

static bool rtc_compile(const std::string& text, std::string* code_object, std::string* log) {
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, text.c_str(), "kf_generated.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof kOpts / sizeof kOpts[0]), kOpts);
    size_t lsz = 0;
    hiprtcGetProgramLogSize(prog, &lsz);
    std::string lg(lsz, '\0');
    if (lsz) hiprtcGetProgramLog(prog, &lg[0]);
    if (r != HIPRTC_SUCCESS) {
        *log = std::string("hipRTC: ") + hiprtcGetErrorString(r) + "\n" + lg;
        if (const char* dump = std::getenv("KF_DUMP_FAILED_SOURCE")) {
            FILE* f = std::fopen(dump, "w");
            if (f) {
                std::fwrite(text.data(), 1, text.size(), f);
                std::fclose(f);
            }
        }
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t csz = 0;
    hiprtcGetCodeSize(prog, &csz);
    code_object->assign(csz, '\0');
    hiprtcGetCode(prog, &(*code_object)[0]);
    hiprtcDestroyProgram(&prog);
    *log = lg;
    return true;
}

std::string jit_cache_ident(const KernelCode& k) {
    const std::string path = cache_path(unit_text(k));
    if (path.empty()) return "";
    struct stat st;
    if (::stat(path.c_str(), &st) != 0) return "";
    return "ino:" + std::to_string((unsigned long long)st.st_dev) + ":" + std::to_string((unsigned long long)st.st_ino);
}

bool jit_compile_one(const KernelCode& k, std::string* code_object, std::string* log) {
    const std::string text = unit_text(k);
    const std::string path = cache_path(text);
    if (!path.empty() && read_file(path, code_object)) return true;
    if (!rtc_compile(text, code_object, log)) return false;
    if (!path.empty()) write_file_atomic(path, with_header(*code_object));
    return true;
}

}  // namespace kf

namespace kf {

bool jit_compile_together(const std::vector<const KernelCode*>& ks, std::string* code_object, std::string* log) {
    std::string text = blocks_source() + "\n";
    for (const KernelCode* k : ks) text += k->source + "\n";
    if (const char* extra = std::getenv("KF_JIT_EXTRA_SOURCE")) text += std::string(extra) + "\n";
    return rtc_compile(text, code_object, log);
}

bool jit_cache_enabled() { return !cache_dir().empty(); }

bool jit_precompile(const std::vector<const KernelCode*>& ks, std::string* log) {
    std::vector<const KernelCode*> todo;
    std::vector<std::string> paths;
    std::string dummy;
    for (const KernelCode* k : ks) {
        std::string path = cache_path(unit_text(*k));
        if (path.empty()) {
            *log = "KF_CACHE_DIR is not set";
            return false;
        }
        std::string have;
        if (read_file(path, &have)) continue;
        bool dup = false;
        for (const std::string& q : paths)
            if (q == path) dup = true;
        if (dup) continue;
        todo.push_back(k);
        paths.push_back(path);
    }
    if (todo.empty()) return true;
    std::string text = blocks_source() + "\n";
    for (const KernelCode* k : todo) text += k->source + "\n";
    if (const char* extra = std::getenv("KF_JIT_EXTRA_SOURCE")) text += std::string(extra) + "\n";
    std::string co;
    if (!rtc_compile(text, &co, log)) return false;
    // one shared code object; every kernel's cache entry links to it
    std::string batch = paths[0] + ".batch";
    const std::string stored = with_header(co);
    write_file_atomic(batch, stored);
    for (const std::string& q : paths) {
        std::remove(q.c_str());
        if (::link(batch.c_str(), q.c_str()) != 0) write_file_atomic(q, stored);
    }
    std::remove(batch.c_str());
    return true;
}

}  // namespace kf
