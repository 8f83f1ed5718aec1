// Generated per-code decode kernels: the unrolled decoder of Sec. III-B, a
// decoder specialised to one frozen set with no run-time schedule, written
// as the list of node-function calls of Listing 1 (Sec. III-B.1) with every
// size and offset a compile-time constant (Sec. III-B.4).
//
// The device schedule of a code is written out as a straight sequence of
// op calls, each with its op word as a literal, into a small HIP source
// that includes the same op library as the schedule-interpreting kernel
// (decode_ops.h).  With every op argument a constant the compiler removes
// all dispatch, folds the output bookkeeping and keeps every node size and
// offset static, so the kernel does the same arithmetic in the same order as
// the interpreter, without its per-op cost.
//
// Compiled code objects are cached on disk under a key that hashes the
// source, the compile options and the compiler version, so a code is
// compiled once per machine image; polar_build_kernel() fills the cache
// ahead of time without a device.
#include <dlfcn.h>
#include <hip/hip_runtime_api.h>
#include <hip/hiprtc.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <string>
#include <vector>

#include "embedded_headers.inc"  // kOpcodesH, kDecodeOpsH: the op library as text
#include "unrolled.h"

namespace polar {

namespace {

const char* const kOptions[] = {"--offload-arch=gfx950", "-mwavefrontsize64", "-O3", "-std=c++17", "-ffp-contract=off",
                                "-fno-honor-nans", "-fno-honor-infinities", "-Xclang", "-target-feature",
                                "-Xclang", "-packed-fp32-ops"};
constexpr int kNumOptions = sizeof(kOptions) / sizeof(kOptions[0]);

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

std::string library_dir() {
  Dl_info info;
  if (dladdr((void*)&library_dir, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t s = p.rfind('/');
    if (s != std::string::npos) return p.substr(0, s);
  }
  return ".";
}

std::string cache_dir() {
  const char* env = getenv("POLAR_KERNEL_CACHE");
  if (env && *env) return env;
  return library_dir() + "/kernels";
}

bool read_file(const std::string& path, std::vector<char>& out) {
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) return false;
  fseek(f, 0, SEEK_END);
  const long sz = ftell(f);
  fseek(f, 0, SEEK_SET);
  out.resize(sz > 0 ? (size_t)sz : 0);
  const bool ok = sz > 0 && fread(out.data(), 1, out.size(), f) == out.size();
  fclose(f);
  return ok;
}

bool write_file_atomic(const std::string& path, const std::vector<char>& data) {
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  const bool ok = fwrite(data.data(), 1, data.size(), f) == data.size();
  if (fclose(f) != 0 || !ok) {
    unlink(tmp.c_str());
    return false;
  }
  if (rename(tmp.c_str(), path.c_str()) != 0) {
    unlink(tmp.c_str());
    return false;
  }
  return true;
}

}  // namespace

namespace {

// The virtual top stage needs both children of the root to be inner nodes
// (or Rate-0): no decision node of size N or N/2.
bool vtop_allowed(const Plan& p) {
  for (int i = 0; i < p.nops; ++i) {
    const unsigned code = p.dops[i] & 0xffu, st = (p.dops[i] >> 8) & 0xffu;
    if ((st == (unsigned)p.log2n || st == (unsigned)p.log2n - 1) && code >= DOP_R1 && code <= DOP_SPC) return false;
  }
  return true;
}

// The stage below the float register stage (N = 32768: stage 12) can be
// virtual when every op on its nodes is f, g, g_0R, a combine, or a Rate-1
// or SPC leaf (the decoder recomputes those from the register stage).
bool vmid_allowed(const Plan& p) {
  if (p.log2n != 15) return false;
  for (int i = 0; i < p.nops; ++i) {
    const unsigned code = p.dops[i] & 0xffu, st = (p.dops[i] >> 8) & 0xffu;
    if (st == (unsigned)p.log2n - 3 && !(code <= DOP_CR0 || code == DOP_R1 || code == DOP_SPC)) return false;
  }
  return true;
}

// The default rule: int8 keeps 2 (N = 32768, below a virtual top stage when
// allowed) or 1 (N = 16384) stages in registers; float codes of N >= 16384
// use the virtual top stage and one register stage when allowed, and at
// N = 32768 the virtual stage below it (a 20 KB slot: two frames per SIMD).
UnrolledLayout default_layout(const Plan& p, int llr_type) {
  UnrolledLayout L;
  if (llr_type != 0) {
    if (p.log2n >= 14 && vtop_allowed(p)) L.vtop = L.nreg = 1;
    if (L.vtop && vmid_allowed(p)) L.vmid = 1;
  } else if (p.log2n == 15) {
    L.nreg = 2;
    L.vtop = vtop_allowed(p) ? 1 : 0;
  } else if (p.log2n == 14) {
    L.nreg = 1;
  }
  return L;
}

// What the decoder templates accept: int8 register stages of >= 2^11 LLRs,
// at most 3 (a leaf at a register stage stages its bits in the highest LDS
// stage), a virtual top stage only above a register stage and for N >= 8192;
// float: one register stage below a virtual top stage (N >= 16384), with or
// without (N = 32768) the virtual stage below it, or neither.
bool layout_valid(const Plan& p, int llr_type, UnrolledLayout L) {
  if (L.vtop < 0 || L.vtop > 1 || L.nreg < 0 || L.vmid < 0 || L.vmid > 1) return false;
  if (L.vtop && !vtop_allowed(p)) return false;
  if (L.vmid && (llr_type == 0 || L.vtop != 1 || L.nreg != 1 || !vmid_allowed(p))) return false;
  if (llr_type != 0) return (L.vtop == 0 && L.nreg == 0) || (L.vtop == 1 && L.nreg <= 1 && p.log2n >= 14);
  if (L.nreg == 0) return L.vtop == 0;
  return L.nreg <= 3 && p.log2n - L.vtop - L.nreg >= 11 && (L.vtop == 0 || p.log2n >= 13);
}

}  // namespace

int unrolled_stage_vgprs(const Plan& p, int llr_type, UnrolledLayout L) {
  const int elem = llr_type == 1 ? 4 : 1;
  int regs = 0;
  for (int t = p.log2n - 1 - L.vtop; t > p.log2n - 1 - L.vtop - L.nreg; --t) regs += ((1 << t) * elem) >> 8;
  return regs;
}

std::vector<UnrolledLayout> unrolled_layouts(const Plan& p, int llr_type) {
  std::vector<UnrolledLayout> out;
  out.push_back(default_layout(p, llr_type));
  // {vtop, nreg}.  int8 candidates leave room for the decoder's working set
  // (about 56 VGPRs) at two waves per SIMD or more; layouts of more register
  // stages are compiled for fewer waves per SIMD (kRegWorkingSet below)
  static const int kTryI8[][3] = {{1, 2, 0}, {1, 1, 0}, {1, 3, 0}, {0, 1, 0}, {0, 2, 0}, {0, 3, 0}, {0, 0, 0}};
  static const int kTryF32[][3] = {{1, 1, 1}, {1, 1, 0}, {1, 0, 0}, {0, 0, 0}};
  const int ntry = llr_type != 0 ? 4 : 7;
  for (int i = 0; i < ntry && out.size() < 6; ++i) {
    const int* t = llr_type != 0 ? kTryF32[i] : kTryI8[i];
    UnrolledLayout L;
    L.vtop = t[0];
    L.nreg = t[1];
    L.vmid = t[2];
    if (!layout_valid(p, llr_type, L)) continue;
    if (llr_type == 0 && unrolled_stage_vgprs(p, llr_type, L) + kRegWorkingSet > 256) continue;
    bool dup = false;
    for (const UnrolledLayout& o : out) dup = dup || (o.vtop == L.vtop && o.nreg == L.nreg && o.vmid == L.vmid);
    if (!dup) out.push_back(L);
  }
  return out;
}

UnrolledLayout unrolled_layout(const Plan& p, int llr_type) {
  if (p.layout > 0) {
    const std::vector<UnrolledLayout> all = unrolled_layouts(p, llr_type);
    if (p.layout < (int)all.size()) return all[(size_t)p.layout];
  }
  return default_layout(p, llr_type);
}

int unrolled_wave_bytes(const Plan& p, int llr_type) {
  const UnrolledLayout L = unrolled_layout(p, llr_type);
  return wave_lds_bytes(p.log2n, llr_type == 1 ? 4 : 1, L.off_lds());
}

int unrolled_waves_per_simd(const Plan& p, int llr_type) {
  // what the LDS slot allows (160 KB per CU, 4 SIMDs) ...
  int w = (160 * 1024 / unrolled_wave_bytes(p, llr_type)) / 4;
  // ... and, for int8, what the register stages leave room for
  if (llr_type == 0) {
    const int regs = unrolled_stage_vgprs(p, llr_type, unrolled_layout(p, llr_type));
    const int wr = 512 / (regs + kRegWorkingSet);
    if (wr < w) w = wr;
  }
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

namespace {


// The decoder object and its initialisation for one code.
std::string decoder_decl(const Plan& p, int llr_type, const char* frame_expr, const char* trace_expr) {
  const UnrolledLayout L = unrolled_layout(p, llr_type);
  const char* pol = llr_type == 1 ? "PF32" : "PI8";
  std::string s;
  s += "  polar::DecU<polar::" + std::string(pol) + ", " + std::to_string(p.log2n) + ", " + std::to_string(L.nreg) +
       ", " + std::to_string(L.vtop) + ", " + std::to_string(L.vmid) + "> d;\n";
  s += "  d.init(base, lane, " + std::to_string(p.log2n) + ", " + std::to_string(p.k) + ", llr, " + frame_expr +
       ", bits, " + trace_expr + ", " + std::to_string(L.off_lds()) + ");\n";
  return s;
}

// Rough vector-instruction cost of one op (int8 kernels; a fit of the
// generated code's instruction counts), used only to place the priority
// steps below.
double op_cost(unsigned code, int st, bool fused) {
  const double size = (double)(1u << st);
  if (fused) return (code == DOP_F ? 0.075 : 0.085) * size;
  if (st <= kRegStages) {
    static const double small[] = {5.0, 1.5, 3.7, 0.6, 1.4, 1.0, 2.0, 2.0, 20.0, 1.4, 0.0, 6.0, 24.0, 28.0, 10.0};
    return code <= DOP_REPR1 ? small[code] : 0.0;
  }
  switch (code) {
    case DOP_F: return 2.0 + 0.025 * size;
    case DOP_G: case DOP_G0R: return 2.0 + 0.028 * size;
    case DOP_R1: return 55.0 + 0.035 * size;
    case DOP_REP: return 20.0 + 0.08 * size;
    case DOP_SPC: return 80.0 + 0.15 * size;
    default: return 2.0 + 0.0006 * size;
  }
}

// The op calls of one code.  With the virtual top stage the root's f / g /
// g_0R emit nothing and the ops of its children become fused ops.
//
// Progress priority: the decoder starts at wave priority 3 and steps down to
// 2, 1 and 0 after 40%, 65% and 85% of its estimated work.  The waves that
// share a SIMD then keep pace with each other (a wave that runs ahead yields
// issue slots to the ones behind) instead of the oldest finishing first and
// the last running alone, with too few waves to hide its latencies.
void append_ops(std::string& s, const Plan& p, int llr_type) {
  const UnrolledLayout L = unrolled_layout(p, llr_type);
  std::vector<double> cost((size_t)p.nops, 0.0);
  double total = 0.0;
  for (int i = 0; i < p.nops; ++i) {
    const unsigned code = p.dops[i] & 0xffu;
    const int st = (int)((p.dops[i] >> 8) & 0xffu);
    if (L.vtop && st == p.log2n && code <= DOP_G0R) continue;
    if (L.vmid && st == p.log2n - 2 && code <= DOP_G0R) continue;
    const bool fused = code <= DOP_G0R && ((L.vtop && st == p.log2n - 1) || (L.vmid && st == p.log2n - 3));
    cost[(size_t)i] = op_cost(code, st, fused);
    total += cost[(size_t)i];
  }
  static const double kSteps[3] = {0.40, 0.65, 0.85};
  int next = 0;
  double done = 0.0;
  char line[96];
  s += "  __builtin_amdgcn_s_setprio(3);\n";
  // with vtop, the root's f / g / g_0R emit nothing and the ops of its
  // children become fused ops; with vmid, likewise the ops of the register
  // stage's nodes and of their children (f / g / g_0R and Rate-1 / SPC
  // leaves, which recompute their LLRs with the parent's op)
  unsigned root_op = DOP_F, mid_op = DOP_F;
  for (int i = 0; i < p.nops; ++i) {
    const unsigned w = p.dops[i];
    const unsigned code = w & 0xffu;
    const int st = (int)((w >> 8) & 0xffu);
    if (L.vtop && st == p.log2n && code <= DOP_G0R) {
      root_op = code;
      continue;
    }
    if (L.vmid && st == p.log2n - 2 && code <= DOP_G0R) {
      mid_op = code;
      continue;
    }
    if (L.vtop && st == p.log2n - 1 && code <= DOP_G0R)
      snprintf(line, sizeof line, "  d.template step_fused<0x%08xu, %uu>();\n", w, root_op);
    else if (L.vmid && st == p.log2n - 3 && (code <= DOP_G0R || code == DOP_R1 || code == DOP_SPC))
      snprintf(line, sizeof line, "  d.template step_mid<0x%08xu, %uu>();\n", w, mid_op);
    else
      snprintf(line, sizeof line, "  d.template step_c<0x%08xu>();\n", w);
    s += line;
    done += cost[(size_t)i];
    while (next < 3 && done >= kSteps[next] * total) {
      snprintf(line, sizeof line, "  __builtin_amdgcn_s_setprio(%d);\n", 2 - next);
      s += line;
      ++next;
    }
  }
}

}  // namespace

std::string unrolled_source(const Plan& p, int llr_type) {
  const char* chan = llr_type == 1 ? "float" : "int8_t";
  const int wps = unrolled_waves_per_simd(p, llr_type);
  std::string s;
  s.reserve(64 * (size_t)p.nops + 4096);
  s += "// generated: unrolled decoder for one polar code\n";
  s += "// N=" + std::to_string(p.n) + " K=" + std::to_string(p.k) + " algo=" + std::to_string(p.algo) +
       " llr=" + std::to_string(llr_type) + " ops=" + std::to_string(p.nops) + "\n";
  s += "#include \"decode_ops.h\"\n\nnamespace {\n\n";
  s += "__device__ __forceinline__ void entry(const " + std::string(chan) + "* llr, int nframes, uint8_t* bits, " +
       chan + "* trace, int wave_bytes, unsigned char* smem) {\n";
  s += "  const int lane = threadIdx.x & 63;\n";
  s += "  const int wid = (int)polar::rfl(threadIdx.x >> 6);\n";
  s += "  const int frame = blockIdx.x * (blockDim.x >> 6) + wid;\n";
  s += "  if (frame >= nframes) return;\n";
  s += "  LDS unsigned char* base = (LDS unsigned char*)smem + wid * wave_bytes;\n";
  s += decoder_decl(p, llr_type, "frame", "trace");
  append_ops(s, p, llr_type);
  s += "  d.finish();\n}\n\n}  // namespace\n\n";
  const std::string attrs =
      "__launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(" + std::to_string(wps) + "))) ";
  s += "extern \"C\" __global__ void " + attrs + "polar_unrolled(const " + std::string(chan) +
       "* __restrict__ llr, int nframes, uint8_t* __restrict__ bits, int wave_bytes) {\n";
  s += "  extern __shared__ __align__(16) unsigned char smem[];\n";
  s += "  entry(llr, nframes, bits, nullptr, wave_bytes, smem);\n}\n\n";
  s += "extern \"C\" __global__ void " + attrs + "polar_unrolled_trace(const " + std::string(chan) +
       "* __restrict__ llr, int nframes, uint8_t* __restrict__ bits, " + chan +
       "* __restrict__ trace, int wave_bytes) {\n";
  s += "  extern __shared__ __align__(16) unsigned char smem[];\n";
  s += "  entry(llr, nframes, bits, trace, wave_bytes, smem);\n}\n";
  return s;
}

std::string batch_source(const std::vector<const Plan*>& plans, int llr_type, int waves_per_simd) {
  const char* chan = llr_type == 1 ? "float" : "int8_t";
  std::string s;
  size_t total_ops = 0;
  for (const Plan* p : plans) total_ops += (size_t)p->nops;
  s.reserve(64 * total_ops + 4096 * plans.size() + 4096);
  s += "// generated: persistent batch decoder for " + std::to_string(plans.size()) + " polar codes\n";
  s += "#include \"decode_ops.h\"\n\nnamespace {\n\n";
  for (size_t c = 0; c < plans.size(); ++c) {
    const Plan& p = *plans[c];
    s += "// code " + std::to_string(c) + ": N=" + std::to_string(p.n) + " K=" + std::to_string(p.k) +
         " algo=" + std::to_string(p.algo) + "\n";
    s += "__device__ __noinline__ void dec_" + std::to_string(c) + "(LDS unsigned char* base, int lane, const " +
         chan + "* llr, uint8_t* bits) {\n";
    s += decoder_decl(p, llr_type, "0", "nullptr");
    append_ops(s, p, llr_type);
    s += "  d.finish();\n}\n\n";
  }
  s += "}  // namespace\n\n";
  // Frame descriptor: two 64-bit words, [0] = code index | bits byte offset << 8,
  // [1] = LLR offset in elements; both offsets signed.  Each wave takes
  // frames wave, wave + W, ...
  s += "extern \"C\" __global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(" +
       std::to_string(waves_per_simd) + "))) polar_batch(const unsigned long long* __restrict__ desc, int nframes, const " +
       chan + "* __restrict__ llr, uint8_t* __restrict__ bits, int wave_bytes) {\n";
  s += "  extern __shared__ __align__(16) unsigned char smem[];\n";
  s += "  const int lane = threadIdx.x & 63;\n";
  s += "  const int wid = (int)polar::rfl(threadIdx.x >> 6);\n";
  s += "  LDS unsigned char* base = (LDS unsigned char*)smem + wid * wave_bytes;\n";
  s += "  const int stride = gridDim.x * (blockDim.x >> 6);\n";
  s += "  for (int f = blockIdx.x * (blockDim.x >> 6) + wid; f < nframes; f += stride) {\n";
  s += "    const unsigned long long d0 = desc[2 * f], d1 = desc[2 * f + 1];\n";
  s += "    switch ((unsigned)(d0 & 255u)) {\n";
  for (size_t c = 0; c < plans.size(); ++c)
    s += "      case " + std::to_string(c) + ": dec_" + std::to_string(c) +
         "(base, lane, llr + (long long)d1, bits + ((long long)d0 >> 8)); break;\n";
  s += "      default: break;\n    }\n  }\n}\n";
  return s;
}

std::string unrolled_cache_path(const std::string& src) {
  uint64_t h = 0xcbf29ce484222325ull;
  h = fnv1a(h, src.data(), src.size());
  h = fnv1a(h, kOpcodesH, sizeof(kOpcodesH));
  h = fnv1a(h, kDecodeOpsH, sizeof(kDecodeOpsH));
  for (int i = 0; i < kNumOptions; ++i) h = fnv1a(h, kOptions[i], strlen(kOptions[i]) + 1);
  int major = 0, minor = 0;
  (void)hiprtcVersion(&major, &minor);
  h = fnv1a(h, &major, sizeof major);
  h = fnv1a(h, &minor, sizeof minor);
  char name[40];
  snprintf(name, sizeof name, "%016llx.hsaco", (unsigned long long)h);
  return cache_dir() + "/" + name;
}

// Returns 0 and the code object, from the cache or freshly compiled (and
// then stored), or -1 with the compiler log.
int unrolled_code_object(const Plan& p, int llr_type, std::vector<char>& code, std::string& log) {
  return source_code_object(unrolled_source(p, llr_type), code, log);
}

int source_code_object(const std::string& src, std::vector<char>& code, std::string& log) {
  const std::string path = unrolled_cache_path(src);
  if (read_file(path, code)) return 0;
  hiprtcProgram prog;
  const char* headers[] = {kOpcodesH, kDecodeOpsH};
  const char* names[] = {"opcodes.h", "decode_ops.h"};
  if (hiprtcCreateProgram(&prog, src.c_str(), "polar_unrolled.hip", 2, headers, names) != HIPRTC_SUCCESS) {
    log = "hiprtcCreateProgram failed";
    return -1;
  }
  const hiprtcResult r = hiprtcCompileProgram(prog, kNumOptions, kOptions);
  size_t log_size = 0;
  if (hiprtcGetProgramLogSize(prog, &log_size) == HIPRTC_SUCCESS && log_size > 1) {
    log.resize(log_size);
    hiprtcGetProgramLog(prog, &log[0]);
  }
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return -1;
  }
  size_t size = 0;
  hiprtcGetCodeSize(prog, &size);
  code.resize(size);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  if (size == 0) return -1;
  const std::string dir = cache_dir();
  mkdir(dir.c_str(), 0755);  // may exist; a failed store only costs a recompile later
  (void)write_file_atomic(path, code);
  return 0;
}

int batch_load(const std::vector<char>& code, hipModule_t& module, hipFunction_t& fn) {
  if (hipModuleLoadData(&module, code.data()) != hipSuccess) return -1;
  if (hipModuleGetFunction(&fn, module, "polar_batch") != hipSuccess) {
    (void)hipModuleUnload(module);
    module = nullptr;
    return -1;
  }
  return 0;
}

int batch_launch(hipFunction_t fn, const void* desc, int nframes, const void* llr, uint8_t* bits, int wave_bytes,
                 int waves_per_block, int blocks, void* stream) {
  const unsigned lds = (unsigned)wave_bytes * (unsigned)waves_per_block;
  // no more workgroups than the frames need (small batches, server steps)
  const int need = (nframes + waves_per_block - 1) / waves_per_block;
  if (blocks > need) blocks = need;
  void* args[] = {(void*)&desc, (void*)&nframes, (void*)&llr, (void*)&bits, (void*)&wave_bytes};
  return (int)hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, 64u * (unsigned)waves_per_block, 1, 1, lds,
                                    (hipStream_t)stream, args, nullptr);
}

int unrolled_load(const std::vector<char>& code, UnrolledKernel& k) {
  if (hipModuleLoadData(&k.module, code.data()) != hipSuccess) return -1;
  if (hipModuleGetFunction(&k.fn, k.module, "polar_unrolled") != hipSuccess ||
      hipModuleGetFunction(&k.fn_trace, k.module, "polar_unrolled_trace") != hipSuccess) {
    (void)hipModuleUnload(k.module);
    k = UnrolledKernel();
    return -1;
  }
  return 0;
}

void unrolled_unload(UnrolledKernel& k) {
  if (k.module) (void)hipModuleUnload(k.module);
  k = UnrolledKernel();
}

int unrolled_launch(const UnrolledKernel& k, const void* llr, int nframes, uint8_t* bits, void* trace,
                    int waves_per_block, void* stream) {
  int wb = k.wave_bytes;
  const unsigned grid = (unsigned)((nframes + waves_per_block - 1) / waves_per_block);
  const unsigned block = 64u * (unsigned)waves_per_block;
  const unsigned lds = (unsigned)wb * (unsigned)waves_per_block;
  hipError_t e;
  if (trace) {
    void* args[] = {(void*)&llr, (void*)&nframes, (void*)&bits, (void*)&trace, (void*)&wb};
    e = hipModuleLaunchKernel(k.fn_trace, grid, 1, 1, block, 1, 1, lds, (hipStream_t)stream, args, nullptr);
  } else {
    void* args[] = {(void*)&llr, (void*)&nframes, (void*)&bits, (void*)&wb};
    e = hipModuleLaunchKernel(k.fn, grid, 1, 1, block, 1, 1, lds, (hipStream_t)stream, args, nullptr);
  }
  return (int)e;
}

}  // namespace polar
