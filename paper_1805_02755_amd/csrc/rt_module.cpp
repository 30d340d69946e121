// Payloads supplied as source at run time: hipRTC compiles the caller's
// work-item function together with the dispenser's device code (the same
// headers the fixed payloads are built from, embedded at build time) into a
// gfx950 code object holding the persistent kernel and the plain kernel of
// that payload.
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>

#include "kernels.hpp"

#include <cctype>
#include <cstring>

namespace ce {

extern const int kRtHeaderCount;
extern const char* const kRtHeaderNames[];
extern const char* const kRtHeaderTexts[];

namespace {

const char* const kPersistentName = "ce::k_persistent<ce::RtTile>";
const char* const kBareName = "ce::k_bare<ce::RtTile>";
const char* const kDirectName = "ce::k_direct<ce::RtTile>";

bool is_identifier(const char* s) {
  if (!s || !*s || !(std::isalpha((unsigned char)*s) || *s == '_')) return false;
  for (const char* p = s; *p; ++p)
    if (!(std::isalnum((unsigned char)*p) || *p == '_')) return false;
  return std::strlen(s) < 256;
}

}  // namespace

int rt_compile(const char* source, const char* entry, std::string* code, std::string* lowered_p,
               std::string* lowered_b, std::string* lowered_d, std::string* log) {
  // returns 0, -1 (source or entry refused, or a compile error) or -2 (hipRTC failed)
  log->clear();
  if (!source || !is_identifier(entry)) {
    *log = "source must be given and entry must be a C identifier";
    return -1;
  }
  std::string prog = "#define CE_RT_ENTRY ";
  prog += entry;
  prog += "\n#include <stdint.h>\n#include \"coexec.h\"\n#line 1 \"payload.hip\"\n";
  prog += source;
  prog += "\n#include \"rt_tile.hpp\"\n#include \"sched_device.hpp\"\n";
  prog += "template __global__ void ce::k_persistent<ce::RtTile>(ce::RtTile, ce::SchedArgs);\n";
  prog += "template __global__ void ce::k_bare<ce::RtTile>(ce::RtTile, uint64_t);\n";
  prog += "template __global__ void ce::k_direct<ce::RtTile>(ce::RtTile, ce::DirectArgs);\n";
  hiprtcProgram p = nullptr;
  if (hiprtcCreateProgram(&p, prog.c_str(), "runtime_payload.hip", kRtHeaderCount, kRtHeaderTexts, kRtHeaderNames) !=
      HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return -2;
  }
  hiprtcAddNameExpression(p, kPersistentName);
  hiprtcAddNameExpression(p, kBareName);
  hiprtcAddNameExpression(p, kDirectName);
  // the options every device file of the library is built with
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(p, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t n = 0;
  if (hiprtcGetProgramLogSize(p, &n) == HIPRTC_SUCCESS && n > 1) {
    log->resize(n);
    hiprtcGetProgramLog(p, &(*log)[0]);
    log->resize(std::strlen(log->c_str()));
  }
  int rc = 0;
  if (r != HIPRTC_SUCCESS) {
    if (log->empty()) *log = hiprtcGetErrorString(r);
    rc = -1;
  } else {
    const char* lp = nullptr;
    const char* lb = nullptr;
    const char* ld = nullptr;
    size_t cs = 0;
    if (hiprtcGetLoweredName(p, kPersistentName, &lp) != HIPRTC_SUCCESS ||
        hiprtcGetLoweredName(p, kBareName, &lb) != HIPRTC_SUCCESS ||
        hiprtcGetLoweredName(p, kDirectName, &ld) != HIPRTC_SUCCESS || hiprtcGetCodeSize(p, &cs) != HIPRTC_SUCCESS ||
        cs == 0) {
      *log += "\nno code object for the runtime payload";
      rc = -2;
    } else {
      *lowered_p = lp;
      *lowered_b = lb;
      *lowered_d = ld;
      code->assign(cs, '\0');
      if (hiprtcGetCode(p, &(*code)[0]) != HIPRTC_SUCCESS) rc = -2;
    }
  }
  hiprtcDestroyProgram(&p);
  return rc;
}

int rt_build(const char* source, const char* entry, void** module, void** fn_persistent, void** fn_bare,
             void** fn_direct, std::string* log) {
  *module = *fn_persistent = *fn_bare = *fn_direct = nullptr;
  std::string code, lp, lb, ld;
  const int rc = rt_compile(source, entry, &code, &lp, &lb, &ld, log);
  if (rc != 0) return rc;
  hipModule_t mod = nullptr;
  hipFunction_t fp = nullptr, fb = nullptr, fd = nullptr;
  if (hipModuleLoadData(&mod, code.data()) != hipSuccess) {
    *log += "\nhipModuleLoadData failed";
    return -3;
  }
  if (hipModuleGetFunction(&fp, mod, lp.c_str()) != hipSuccess || hipModuleGetFunction(&fb, mod, lb.c_str()) != hipSuccess ||
      hipModuleGetFunction(&fd, mod, ld.c_str()) != hipSuccess) {
    (void)hipModuleUnload(mod);
    *log += "\nhipModuleGetFunction failed";
    return -3;
  }
  *module = mod;
  *fn_persistent = fp;
  *fn_bare = fb;
  *fn_direct = fd;
  return 0;
}

void rt_release(void* module) {
  if (module) (void)hipModuleUnload((hipModule_t)module);
}

}  // namespace ce
