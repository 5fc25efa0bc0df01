// The driver-compilation cache of generated kernel source (see fx_jit.hpp).
#include <hip/hiprtc.h>

#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fx_core.hpp"
#include "fx_jit.hpp"

namespace fx {

struct jit_program {
  std::vector<char> code;
  std::map<std::pair<int, std::string>, hipFunction_t> fns;  // (device, name)
  std::map<int, hipModule_t> modules;                         // per device
};

namespace {

std::mutex& jit_mutex() {
  static std::mutex m;
  return m;
}
std::map<std::string, jit_program*>& jit_cache() {
  static std::map<std::string, jit_program*> c;  // entries live until the process ends
  return c;
}

int compile(const std::string& src, std::vector<char>& code) {
  hiprtcProgram p;
  if (hiprtcCreateProgram(&p, src.c_str(), "fx_generated.hip", 0, nullptr, nullptr) !=
      HIPRTC_SUCCESS)
    return fail(FX_E_HIP, "hiprtcCreateProgram failed");
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(p, 6, opts);
  std::string log;
  size_t ls = 0;
  hiprtcGetProgramLogSize(p, &ls);
  if (ls > 1) {
    log.resize(ls);
    hiprtcGetProgramLog(p, &log[0]);
  }
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&p);
    return fail(FX_E_HIP, "hipRTC compilation failed (%s): %.400s", hiprtcGetErrorString(r),
                log.c_str());
  }
  size_t cs = 0;
  hiprtcGetCodeSize(p, &cs);
  code.resize(cs);
  hiprtcGetCode(p, code.data());
  hiprtcDestroyProgram(&p);
  return FX_OK;
}

}  // namespace

int jit_obtain(const char* src, size_t len, jit_program** prog, double* compile_ms) {
  if (!src || !prog) return fail(FX_E_ARG, "NULL argument");
  if (compile_ms) *compile_ms = 0;
  std::string key(src, len);
  std::lock_guard<std::mutex> g(jit_mutex());
  auto it = jit_cache().find(key);
  if (it == jit_cache().end()) {
    jit_program* p = new (std::nothrow) jit_program;
    if (!p) return fail(FX_E_ARG, "out of host memory");
    const auto t0 = std::chrono::steady_clock::now();
    if (int rc = compile(key, p->code)) {
      delete p;
      return rc;
    }
    if (compile_ms)
      *compile_ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    it = jit_cache().emplace(std::move(key), p).first;
  }
  *prog = it->second;
  return FX_OK;
}

int jit_function(jit_program* prog, const char* name, hipFunction_t* fn) {
  if (!prog || !name || !fn) return fail(FX_E_ARG, "NULL argument");
  int dev = 0;
  if (int rc = hip_check(hipGetDevice(&dev), "hipGetDevice")) return rc;
  std::lock_guard<std::mutex> g(jit_mutex());
  auto f = prog->fns.find({dev, name});
  if (f != prog->fns.end()) {
    *fn = f->second;
    return FX_OK;
  }
  auto m = prog->modules.find(dev);
  if (m == prog->modules.end()) {
    hipModule_t mod;
    if (int rc = hip_check(hipModuleLoadData(&mod, prog->code.data()), "hipModuleLoadData"))
      return rc;
    m = prog->modules.emplace(dev, mod).first;
  }
  hipFunction_t h;
  if (int rc = hip_check(hipModuleGetFunction(&h, m->second, name), name)) return rc;
  prog->fns.emplace(std::make_pair(dev, std::string(name)), h);
  *fn = h;
  return FX_OK;
}

int jit_launch(hipFunction_t f, int64_t gx, int64_t gy, int block, void** args, hipStream_t st) {
  if (gx <= 0 || gy <= 0 || gx > 0x7fffffff || gy > 65535)
    return fail(FX_E_UNSUPPORTED, "grid %lld x %lld outside the launch limits", (long long)gx,
                (long long)gy);
  return hip_check(hipModuleLaunchKernel(f, (unsigned)gx, (unsigned)gy, 1, (unsigned)block, 1, 1, 0,
                                         st, args, nullptr),
                   "generated kernel launch");
}

}  // namespace fx
