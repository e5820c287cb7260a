// Run-time specialisation of the per-order kernels for orders 13..15, the
// analogue of the paper's jit clause (Sec. IV): the order, known only when a
// mesh is set up, becomes a compile-time constant of generated code, as it is
// in the kernels the library is built with.
//
// The source is the library's own kernel headers (sem_kernels.h and what it
// includes), embedded at build time, so the run-time kernels are the built
// kernels instantiated for another order.  hipRTC compiles them for the
// device's architecture with the library's compile flags; the code object is
// kept in memory per (architecture, order, runtime version) and written to a
// disk cache, the module is loaded once per device, and launches use the
// grids and work-group sizes of the built launchers.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <sys/stat.h>
#include <unistd.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "sem_internal.h"
#include "sem_kernels.h"
#include "sem_rtc.h"
#include "sem_rtc_headers.inc"

namespace semk {

namespace {

// hipRTC supplies the device runtime itself; the standard headers our
// kernel headers include are given as these stand-ins.
const char kRtcStdint[] =
    "#pragma once\n"
    "typedef __hip_internal::int8_t int8_t;\n"
    "typedef __hip_internal::int16_t int16_t;\n"
    "typedef __hip_internal::int32_t int32_t;\n"
    "typedef __hip_internal::int64_t int64_t;\n"
    "typedef __hip_internal::uint8_t uint8_t;\n"
    "typedef __hip_internal::uint16_t uint16_t;\n"
    "typedef __hip_internal::uint32_t uint32_t;\n"
    "typedef __hip_internal::uint64_t uint64_t;\n"
    "#ifndef INT32_MAX\n#define INT32_MAX 2147483647\n#endif\n";
const char kRtcMath[] =
    "#pragma once\n"
    "#ifndef M_PI\n#define M_PI 3.14159265358979323846\n#endif\n";
const char kRtcEmpty[] = "#pragma once\n";

enum RtcKernel {
  kRtcSetupGeom,
  kRtcAx,
  kRtcAxCg,
  kRtcGatherAssembled,
  kRtcGatherMasked,
  kRtcGatherInverse,
  kRtcCgInit,
  kRtcCgUpdate,
  kRtcFillC,
  kRtcCount
};

std::string name_expression(int k, int N1) {
  const std::string n = std::to_string(N1);
  switch (k) {
    case kRtcSetupGeom: return "&semk::setup_geom_kernel<" + n + ">";
    case kRtcAx: return "&semk::ax_mfma_kernel<" + n + ", semk::PrecF64, false>";
    case kRtcAxCg: return "&semk::ax_mfma_kernel<" + n + ", semk::PrecF64, true>";
    case kRtcGatherAssembled: return "&semk::gather_kernel<" + n + ", 0, double>";
    case kRtcGatherMasked: return "&semk::gather_kernel<" + n + ", 1, double>";
    case kRtcGatherInverse: return "&semk::gather_kernel<" + n + ", 2, double>";
    case kRtcCgInit: return "&semk::cg_init_kernel<" + n + ">";
    case kRtcCgUpdate: return "&semk::cg_update_kernel<" + n + ", double>";
    case kRtcFillC: return "&semk::fill_c_kernel<" + n + ">";
    default: return "";
  }
}
static_assert(kGatherAssembled == 0 && kGatherMasked == 1 && kGatherInverse == 2,
              "gather modes as spelled in the name expressions");

// The program: the kernel header; the name expressions instantiate the
// kernels of one order.
const char kRtcSource[] = "#include \"sem_kernels.h\"\n";

std::vector<std::string> compile_options(const std::string &arch) {
  // the flags of the built kernels (build.py): optimisation, contraction only
  // within one expression, and no packed FP32 instructions
  return {"--offload-arch=" + arch, "-O3", "-std=c++17", "-ffp-contract=on",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
}

struct Code {
  std::vector<char> bytes;
  std::string lowered[kRtcCount];
};

struct Loaded {
  hipModule_t mod = nullptr;
  hipFunction_t fn[kRtcCount] = {};
};

std::mutex g_mu;
std::map<std::string, Code> g_code;                // key -> code object
std::map<std::pair<int, int>, Loaded> g_loaded;    // (device, order) -> module

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
  const unsigned char *c = (const unsigned char *)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Cache key: every source text, the options, the order, the architecture
// and the compiler and runtime versions.
std::string cache_key(int N, const std::string &arch) {
  uint64_t h = 1469598103934665603ull;
  for (int i = 0; i < kRtcHeaderCount; ++i) {
    h = fnv1a(h, kRtcHeaderNames[i], std::strlen(kRtcHeaderNames[i]) + 1);
    h = fnv1a(h, kRtcHeaderTexts[i], std::strlen(kRtcHeaderTexts[i]) + 1);
  }
  h = fnv1a(h, kRtcSource, sizeof(kRtcSource));
  for (const std::string &o : compile_options(arch)) h = fnv1a(h, o.c_str(), o.size() + 1);
  int major = 0, minor = 0, rt = 0;
  (void)hiprtcVersion(&major, &minor);
  (void)hipRuntimeGetVersion(&rt);
  const int v[4] = {N, major, minor, rt};
  h = fnv1a(h, v, sizeof(v));
  char buf[96];
  std::snprintf(buf, sizeof(buf), "%s_N%d_%016llx", arch.c_str(), N, (unsigned long long)h);
  return buf;
}

// Directory of the disk cache: $SEM_RTC_CACHE, else $XDG_CACHE_HOME/libsem,
// else $HOME/.cache/libsem; "" when none is usable.
std::string cache_dir() {
  std::string d;
  if (const char *e = std::getenv("SEM_RTC_CACHE")) {
    d = e;
  } else if (const char *x = std::getenv("XDG_CACHE_HOME")) {
    d = std::string(x) + "/libsem";
  } else if (const char *hm = std::getenv("HOME")) {
    d = std::string(hm) + "/.cache";
    (void)mkdir(d.c_str(), 0755);
    d += "/libsem";
  } else {
    return "";
  }
  (void)mkdir(d.c_str(), 0755);
  return access(d.c_str(), W_OK | R_OK) == 0 ? d : "";
}

bool read_cached(const std::string &dir, const std::string &key, Code *c) {
  if (dir.empty()) return false;
  FILE *f = std::fopen((dir + "/" + key + ".co").c_str(), "rb");
  if (!f) return false;
  std::vector<char> bytes;
  char buf[1 << 16];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) bytes.insert(bytes.end(), buf, buf + got);
  std::fclose(f);
  FILE *g = std::fopen((dir + "/" + key + ".names").c_str(), "r");
  if (!g) return false;
  Code out;
  char line[4096];
  int k = 0;
  while (k < kRtcCount && std::fgets(line, sizeof(line), g)) {
    std::string s(line);
    while (!s.empty() && (s.back() == '\n' || s.back() == '\r')) s.pop_back();
    out.lowered[k++] = s;
  }
  std::fclose(g);
  if (k != kRtcCount || bytes.empty()) return false;
  out.bytes = std::move(bytes);
  *c = std::move(out);
  return true;
}

void write_cached(const std::string &dir, const std::string &key, const Code &c) {
  if (dir.empty()) return;
  // write under temporary names, then rename: readers never see a partial file
  const std::string tmp = dir + "/" + key + ".tmp" + std::to_string((long)getpid());
  FILE *f = std::fopen((tmp + ".co").c_str(), "wb");
  if (!f) return;
  const bool ok_co = std::fwrite(c.bytes.data(), 1, c.bytes.size(), f) == c.bytes.size();
  std::fclose(f);
  FILE *g = std::fopen((tmp + ".names").c_str(), "w");
  if (!g) return;
  bool ok_n = true;
  for (int k = 0; k < kRtcCount; ++k) ok_n = ok_n && std::fprintf(g, "%s\n", c.lowered[k].c_str()) > 0;
  std::fclose(g);
  if (ok_co && ok_n) {
    (void)std::rename((tmp + ".names").c_str(), (dir + "/" + key + ".names").c_str());
    (void)std::rename((tmp + ".co").c_str(), (dir + "/" + key + ".co").c_str());
  } else {
    (void)std::remove((tmp + ".co").c_str());
    (void)std::remove((tmp + ".names").c_str());
  }
}

// Compile the kernels of order N for `arch` (g_mu held).
hipError_t compile(int N, const std::string &arch, Code *out, std::string *why) {
  std::vector<const char *> hdr_texts, hdr_names;
  for (int i = 0; i < kRtcHeaderCount; ++i) {
    hdr_texts.push_back(kRtcHeaderTexts[i]);
    hdr_names.push_back(kRtcHeaderNames[i]);
  }
  const char *stand_in_names[] = {"hip/hip_runtime.h", "cstdint", "stdint.h", "cstddef", "stddef.h", "cmath"};
  const char *stand_in_texts[] = {kRtcMath, kRtcStdint, kRtcStdint, kRtcEmpty, kRtcEmpty, kRtcMath};
  for (int i = 0; i < 6; ++i) {
    hdr_texts.push_back(stand_in_texts[i]);
    hdr_names.push_back(stand_in_names[i]);
  }
  hiprtcProgram prog = nullptr;
  hiprtcResult r = hiprtcCreateProgram(&prog, kRtcSource, "sem_rtc_kernels.hip", (int)hdr_texts.size(),
                                       hdr_texts.data(), hdr_names.data());
  if (r != HIPRTC_SUCCESS) {
    *why = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
    return hipErrorInvalidImage;
  }
  std::string expr[kRtcCount];
  for (int k = 0; k < kRtcCount; ++k) {
    expr[k] = name_expression(k, N + 1);
    (void)hiprtcAddNameExpression(prog, expr[k].c_str());
  }
  const std::vector<std::string> opts = compile_options(arch);
  std::vector<const char *> copts;
  for (const std::string &o : opts) copts.push_back(o.c_str());
  r = hiprtcCompileProgram(prog, (int)copts.size(), copts.data());
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    (void)hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) (void)hiprtcGetProgramLog(prog, &log[0]);
    *why = std::string("hiprtcCompileProgram (order ") + std::to_string(N) + "): " +
           hiprtcGetErrorString(r) + "\n" + log;
    (void)hiprtcDestroyProgram(&prog);
    return hipErrorInvalidImage;
  }
  Code c;
  for (int k = 0; k < kRtcCount; ++k) {
    const char *low = nullptr;
    if (hiprtcGetLoweredName(prog, expr[k].c_str(), &low) != HIPRTC_SUCCESS || !low) {
      *why = "hiprtcGetLoweredName failed for " + expr[k];
      (void)hiprtcDestroyProgram(&prog);
      return hipErrorInvalidImage;
    }
    c.lowered[k] = low;
  }
  size_t bytes = 0;
  (void)hiprtcGetCodeSize(prog, &bytes);
  c.bytes.resize(bytes);
  r = bytes ? hiprtcGetCode(prog, c.bytes.data()) : HIPRTC_ERROR_COMPILATION;
  (void)hiprtcDestroyProgram(&prog);
  if (r != HIPRTC_SUCCESS) {
    *why = "hiprtcGetCode: no code object";
    return hipErrorInvalidImage;
  }
  *out = std::move(c);
  return hipSuccess;
}

// The code object of order N for `arch`: memory, then disk, then compile
// (g_mu held).
hipError_t code_for(int N, const std::string &arch, const Code **out, std::string *why) {
  const std::string key = cache_key(N, arch);
  auto it = g_code.find(key);
  if (it == g_code.end()) {
    Code c;
    const std::string dir = cache_dir();
    if (!read_cached(dir, key, &c)) {
      const hipError_t e = compile(N, arch, &c, why);
      if (e != hipSuccess) return e;
      write_cached(dir, key, c);
    }
    it = g_code.emplace(key, std::move(c)).first;
  }
  *out = &it->second;
  return hipSuccess;
}

// Base architecture name of the current device ("gfx950" of
// "gfx950:sramecc+:xnack-"): the code object is built for any setting of
// the target features, as the library's own kernels are.
hipError_t device_arch(int dev, std::string *arch) {
  hipDeviceProp_t prop;
  const hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return e;
  std::string a(prop.gcnArchName);
  const size_t colon = a.find(':');
  *arch = colon == std::string::npos ? a : a.substr(0, colon);
  return hipSuccess;
}

// The loaded kernel k of order N on the current device (after rtc_prepare).
hipError_t function_for(int N, int k, hipFunction_t *f) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_loaded.find({dev, N});
  if (it == g_loaded.end() || !it->second.fn[k]) return hipErrorNotInitialized;
  *f = it->second.fn[k];
  return hipSuccess;
}

hipError_t launch(int N, int k, dim3 grid, dim3 block, hipStream_t s, void **args) {
  if (grid.x == 0) return hipSuccess;
  hipFunction_t f = nullptr;
  const hipError_t e = function_for(N, k, &f);
  if (e != hipSuccess) return e;
  return hipModuleLaunchKernel(f, grid.x, grid.y, grid.z, block.x, block.y, block.z, 0, s, args,
                               nullptr);
}

// Launch shapes of the built launchers, per order.
struct Shape {
  int setup_epb, setup_threads;  // AxCfg
  int ax_epb, ax_threads;        // MfmaCfg
  int upd_block;                 // UpdTile<N1, double>::BLOCK
};

template <int N1>
Shape shape_of() {
  static_assert(UpdTile<N1, double>::LINEAR, "FP64 update of these orders is the linear tile");
  return {AxCfg<N1>::EPB, AxCfg<N1>::THREADS, MfmaCfg<N1>::EPB, MfmaCfg<N1>::THREADS,
          UpdTile<N1, double>::BLOCK};
}

Shape shape(int N) {
  switch (N) {
    case 13: return shape_of<14>();
    case 14: return shape_of<15>();
    case 15: return shape_of<16>();
    default: return {1, 64, 1, 64, kVecThreads};
  }
}
static_assert(kMaxRtcOrder == 15, "shape() covers every run-time order");

}  // namespace

bool rtc_arch_supported(const char *arch) {
  // the kernels are written for gfx950 (CDNA4 MFMA shapes and LDS size); a
  // feature suffix such as ":sramecc+:xnack-" is allowed
  if (!arch) return false;
  return std::strncmp(arch, "gfx950", 6) == 0 && (arch[6] == '\0' || arch[6] == ':');
}

hipError_t rtc_build(int N, const char *arch, size_t *code_bytes, std::string *why) {
  if (!rtc_order(N)) {
    *why = "order outside the run-time set";
    return hipErrorInvalidValue;
  }
  if (!rtc_arch_supported(arch)) {
    *why = std::string("architecture ") + (arch ? arch : "(null)") + " is not gfx950";
    return hipErrorInvalidDeviceFunction;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  const Code *c = nullptr;
  const hipError_t e = code_for(N, arch, &c, why);
  if (e == hipSuccess && code_bytes) *code_bytes = c->bytes.size();
  return e;
}

hipError_t rtc_prepare(int N, std::string *why) {
  if (!rtc_order(N)) {
    *why = "order outside the run-time set";
    return hipErrorInvalidValue;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_loaded.count({dev, N})) return hipSuccess;
  std::string arch;
  e = device_arch(dev, &arch);
  if (e != hipSuccess) return e;
  if (!rtc_arch_supported(arch.c_str())) {
    *why = "the current device is " + arch + ", not gfx950";
    return hipErrorInvalidDeviceFunction;
  }
  const Code *c = nullptr;
  e = code_for(N, arch, &c, why);
  if (e != hipSuccess) return e;
  Loaded L;
  e = hipModuleLoadData(&L.mod, c->bytes.data());
  if (e != hipSuccess) {
    *why = "hipModuleLoadData of the run-time code object";
    return e;
  }
  for (int k = 0; k < kRtcCount; ++k) {
    e = hipModuleGetFunction(&L.fn[k], L.mod, c->lowered[k].c_str());
    if (e != hipSuccess) {
      *why = "hipModuleGetFunction " + c->lowered[k];
      (void)hipModuleUnload(L.mod);
      return e;
    }
  }
  g_loaded.emplace(std::make_pair(dev, N), L);  // kept until the process ends
  return hipSuccess;
}

hipError_t rtc_setup_geom(const Box &b, double amp, const double *D, const double *nodes, double *G,
                          double *diag, hipStream_t s) {
  const Shape sh = shape(b.N);
  Box bb = b;
  void *args[] = {&bb, &amp, &D, &nodes, &G, &diag};
  return launch(b.N, kRtcSetupGeom, dim3((unsigned)((b.E() + sh.setup_epb - 1) / sh.setup_epb)),
                dim3(sh.setup_threads), s, args);
}

hipError_t rtc_ax_f64(const Box &b, const double *D, const double *G, double *u, double *w,
                      const double *r, const double *minv, double *x, CgState *cg, double *part,
                      hipStream_t s) {
  const Shape sh = shape(b.N);
  int64_t E = b.E();
  void *args[] = {&E, &D, &G, &u, &w, &r, &minv, &x, &cg, &part};
  return launch(b.N, cg ? kRtcAxCg : kRtcAx, dim3((unsigned)((E + sh.ax_epb - 1) / sh.ax_epb)),
                dim3(sh.ax_threads), s, args);
}

hipError_t rtc_gather(const Box &b, const double *wl, double *out, int mode, hipStream_t s) {
  const int k = mode == kGatherAssembled ? kRtcGatherAssembled
                : mode == kGatherMasked  ? kRtcGatherMasked
                : mode == kGatherInverse ? kRtcGatherInverse
                                         : -1;
  if (k < 0) return hipErrorInvalidValue;
  Box bb = b;
  int64_t L = b.L(), nt = vec_num_blocks(L);
  void *args[] = {&bb, &L, &nt, &wl, &out};
  return launch(b.N, k, dim3((unsigned)vec_grid_blocks(L)), dim3(kVecThreads), s, args);
}

hipError_t rtc_cg_init(const Box &b, const double *bvec, double *x, double *r, double *p,
                       const double *minv, double *part_a, double *part_b, hipStream_t s) {
  Box bb = b;
  int64_t L = b.L(), nt = vec_num_blocks(L);
  void *args[] = {&bb, &L, &nt, &bvec, &x, &r, &p, &minv, &part_a, &part_b};
  return launch(b.N, kRtcCgInit, dim3((unsigned)vec_grid_blocks(L)), dim3(kVecThreads), s, args);
}

hipError_t rtc_cg_update(const Box &b, double *r, const double *w, const double *minv, CgState *st,
                         double *part_rr, double *part_rz, hipStream_t s) {
  const Shape sh = shape(b.N);
  Box bb = b;
  int64_t nt = upd_num_tiles(b, true);
  void *args[] = {&bb, &nt, &r, &w, &minv, &st, &part_rr, &part_rz};
  return launch(b.N, kRtcCgUpdate, dim3((unsigned)upd_grid_blocks(b, true)), dim3(sh.upd_block), s,
                args);
}

hipError_t rtc_fill_c(const Box &b, double *c, hipStream_t s) {
  Box bb = b;
  int64_t L = b.L();
  void *args[] = {&bb, &L, &c};
  return launch(b.N, kRtcFillC, dim3((unsigned)vec_num_blocks(L)), dim3(kVecThreads), s, args);
}

}  // namespace semk
