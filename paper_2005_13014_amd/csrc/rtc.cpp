// Run-time compilation of generated stencil kernels (the front end's code
// generation target): HIP source -> hipRTC for gfx950 -> code object ->
// module function.  The front end specialises every kernel on its extents
// and strides (compile-time shapes, Sec. IV), so a program is compiled once
// per shape and launched many times.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <string>
#include <vector>

#include "stencil.h"

#define STENCIL_API extern "C" __attribute__((visibility("default")))

namespace stl {
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
}  // namespace stl

using namespace stl;

namespace {

struct RtcKernel {
    hipModule_t module = nullptr;
    hipFunction_t function = nullptr;
};

}  // namespace

STENCIL_API int stencil_rtc_compile(const char *source, const char *kernel_name, void **handle) {
    if (!source || !kernel_name || !handle) return fail(STENCIL_E_NULL, "rtc_compile: NULL argument");
    *handle = nullptr;
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, source, "stencil_generated.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return fail(STENCIL_E_HIP, "rtc_compile: hiprtcCreateProgram failed");
    // The same code-generation flags as the library's own kernels.
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, static_cast<int>(sizeof(opts) / sizeof(opts[0])), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        if (hiprtcGetProgramLogSize(prog, &n) != HIPRTC_SUCCESS) n = 0;
        std::string log(n + 1, '\0');
        if (n && hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) log = "(no log)";
        hiprtcDestroyProgram(&prog);
        return fail(STENCIL_E_ARG, "rtc_compile: %s", log.c_str());
    }
    size_t size = 0;
    std::vector<char> code;
    bool got = hiprtcGetCodeSize(prog, &size) == HIPRTC_SUCCESS && size > 0;
    if (got) {
        code.resize(size);
        got = hiprtcGetCode(prog, code.data()) == HIPRTC_SUCCESS;
    }
    hiprtcDestroyProgram(&prog);
    if (!got) return fail(STENCIL_E_HIP, "rtc_compile: no code object from hipRTC");

    RtcKernel *k = new RtcKernel;
    hipError_t e = hipModuleLoadData(&k->module, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&k->function, k->module, kernel_name);
    if (e != hipSuccess) {
        if (k->module) hipModuleUnload(k->module);
        delete k;
        return hip_fail(e, "rtc_compile: module load");
    }
    *handle = k;
    return STENCIL_OK;
}

STENCIL_API int stencil_rtc_launch(void *handle, const uint32_t grid[3], const uint32_t block[3], void **args,
                                   void *stream) {
    if (!handle || !grid || !block || !args) return fail(STENCIL_E_NULL, "rtc_launch: NULL argument");
    const RtcKernel *k = static_cast<const RtcKernel *>(handle);
    if (!grid[0] || !grid[1] || !grid[2]) return STENCIL_OK;  // nothing to do
    if (static_cast<uint64_t>(block[0]) * block[1] * block[2] > 1024 || !block[0] || !block[1] || !block[2])
        return fail(STENCIL_E_ARG, "rtc_launch: block of %u x %u x %u threads", block[0], block[1], block[2]);
    const hipError_t e = hipModuleLaunchKernel(k->function, grid[0], grid[1], grid[2], block[0], block[1],
                                               block[2], 0, static_cast<hipStream_t>(stream), args, nullptr);
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "rtc_launch");
}

STENCIL_API int stencil_rtc_release(void *handle) {
    if (!handle) return STENCIL_OK;
    RtcKernel *k = static_cast<RtcKernel *>(handle);
    const hipError_t e = hipModuleUnload(k->module);
    delete k;
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "rtc_release");
}
