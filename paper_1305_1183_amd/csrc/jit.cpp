// jit.cpp -- run-time compilation of generated kernels with hipRTC for gfx950.
//
// The paper's compiler emits CUDA source and hands it to the vendor compiler
// (Section 4.3); here the generated HIP source is compiled in-process by
// hipRTC into a gfx950 code object. All kernels of one request are compiled
// as one translation unit behind the building-block header.
#include <hip/hiprtc.h>
#include <cstdio>

#include <cstdlib>
#include <mutex>

#include "kf_internal.h"

namespace kf {

static const char kBlocksText[] =
#include "kf_blocks_embed.inc"
    ;

const std::string& blocks_source() {
    static const std::string s(kBlocksText);
    return s;
}

bool jit_compile(const std::vector<const KernelCode*>& ks, std::string* code_object,
                 std::string* log) {
    static std::mutex mu;  // hipRTC programs are independent, but keep logs ordered
    std::lock_guard<std::mutex> lock(mu);
    std::string src = blocks_source();
    src += "\n";
    for (const KernelCode* k : ks) {
        src += k->source;
        src += "\n";
    }
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, src.c_str(), "kf_generated.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t lsz = 0;
    hiprtcGetProgramLogSize(prog, &lsz);
    std::string lg(lsz, '\0');
    if (lsz) hiprtcGetProgramLog(prog, &lg[0]);
    if (r != HIPRTC_SUCCESS) {
        *log = std::string("hipRTC: ") + hiprtcGetErrorString(r) + "\n" + lg;
        if (const char* dump = std::getenv("KF_DUMP_FAILED_SOURCE")) {
            FILE* f = std::fopen(dump, "w");
            if (f) { std::fwrite(src.data(), 1, src.size(), f); std::fclose(f); }
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

}  // namespace kf
