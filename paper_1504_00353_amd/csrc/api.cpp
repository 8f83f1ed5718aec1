// C ABI of libpolar: argument validation, status codes, code objects,
// device upload and the host encoder.  See include/polar.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/polar.h"
#include "internal.h"
#include "noalloc.h"

namespace polar {
int launch_decode(const uint32_t* ops, int nops, int log2n, int kbits, int llr_type, const void* llr, int nframes,
                  uint8_t* bits, void* trace, int waves_per_block, void* stream);
int set_lds_limit(int bytes);
}  // namespace polar

namespace polar {

namespace {
// allocations to let through before the armed failure; -1: none armed
std::atomic<long> g_fail_countdown{-1};
}  // namespace

void arm_alloc_failure(int after) { g_fail_countdown.store(after < 0 ? -1 : (long)after); }

bool alloc_fails() {
  long c = g_fail_countdown.load();
  while (c >= 0) {
    if (g_fail_countdown.compare_exchange_weak(c, c - 1)) return c == 0;
  }
  return false;
}

hipError_t dev_malloc(void** p, size_t bytes) {
  if (alloc_fails()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

hipError_t pinned_malloc(void** p, size_t bytes) {
  if (alloc_fails()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  return hipHostMalloc(p, bytes, 0);
}

}  // namespace polar

namespace {

thread_local polar_status g_last = POLAR_OK;
thread_local std::string g_message;

polar_status set(polar_status s) {
  g_last = s;
  if (s == POLAR_OK) g_message.clear();
  return s;
}

polar_status set_msg(polar_status s, const std::string& msg) {
  g_last = s;
  g_message = msg;
  return s;
}

// Kernels of a code or batch are loaded on the device it was prepared on;
// launches go to the caller's current device.
bool on_device(int dev) {
  int cur = -1;
  return hipGetDevice(&cur) == hipSuccess && cur == dev;
}

// LLR buffers: int8 rows on 4-byte boundaries, float rows on 16-byte
// boundaries (the kernels read whole 32-bit and 128-bit words).
bool llr_aligned(int llr_type, const void* p) {
  return ((uintptr_t)p & (llr_type == POLAR_LLR_F32 ? 15u : 3u)) == 0;
}

int log2_exact(int n) {
  if (n < 2 || n > polar::kMaxN || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

polar_code* make_code(int n, std::vector<uint8_t>&& frozen) {
  polar_code* c = polar::alloc_fails() ? nullptr : new (std::nothrow) polar_code;
  if (!c) {
    set(POLAR_ENOMEM);
    return nullptr;
  }
  try {
    c->plan.n = n;
    c->plan.log2n = log2_exact(n);
    c->plan.frozen = std::move(frozen);
    int k = 0;
    for (uint8_t f : c->plan.frozen) k += f ? 0 : 1;
    c->plan.k = k;
    c->plan.algo = POLAR_ALGO_FASTSSC;
    polar::build_schedule(c->plan);
  } catch (const std::bad_alloc&) {
    delete c;
    set(POLAR_ENOMEM);
    return nullptr;
  }
  set(POLAR_OK);
  return c;
}

// Releases what polar_prepare loaded, so the code can be configured and
// prepared again.
void unprepare(polar_code* c) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != c->device) (void)hipSetDevice(c->device);
  if (c->d_ops) (void)hipFree(c->d_ops);
  c->d_ops = nullptr;
  polar::unrolled_unload(c->unrolled);
  if (cur != c->device) (void)hipSetDevice(cur);
  c->prepared = false;
}

}  // namespace

polar_status polar_set_status(polar_status s) { return set(s); }

extern "C" {

polar_code* polar_construct(int n, int k, double design_ebn0_db) {
  if (log2_exact(n) < 0 || k < 1 || k > n) {
    set(POLAR_EINVAL);
    return nullptr;
  }
  std::vector<uint8_t> frozen;
  if (!polar::construct_frozen(n, k, design_ebn0_db, frozen)) {
    set(POLAR_EINVAL);
    return nullptr;
  }
  return make_code(n, std::move(frozen));
}

polar_code* polar_construct_mask(int n, const uint8_t* frozen) {
  if (log2_exact(n) < 0 || !frozen) {
    set(POLAR_EINVAL);
    return nullptr;
  }
  std::vector<uint8_t> f(frozen, frozen + n);
  int k = 0;
  for (uint8_t v : f) {
    if (v > 1) {
      set(POLAR_EINVAL);
      return nullptr;
    }
    k += v ? 0 : 1;
  }
  if (k < 1) {
    set(POLAR_EINVAL);
    return nullptr;
  }
  return make_code(n, std::move(f));
}

polar_status polar_configure(polar_code* c, polar_algo algo, polar_llr llr_type) {
  if (!c) return set(POLAR_EINVAL);
  if (c->prepared) return set(POLAR_ESTATE);
  if ((algo != POLAR_ALGO_FASTSSC && algo != POLAR_ALGO_SC) || (llr_type != POLAR_LLR_I8 && llr_type != POLAR_LLR_F32))
    return set(POLAR_EINVAL);
  try {
    c->plan.algo = algo;
    c->llr_type = llr_type;
    c->plan.layout = 0;  // the candidates depend on the LLR type and the schedule
    polar::build_schedule(c->plan);
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  return set(POLAR_OK);
}

polar_status polar_set_fused_nodes(polar_code* c, int enable) {
  if (!c) return set(POLAR_EINVAL);
  if (c->prepared) return set(POLAR_ESTATE);
  if (enable != 0 && enable != 1) return set(POLAR_EINVAL);
  try {
    c->plan.fuse = enable;
    c->plan.layout = 0;
    polar::build_schedule(c->plan);
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  return set(POLAR_OK);
}

int polar_layout_count(const polar_code* c) {
  if (!c) {
    set(POLAR_EINVAL);
    return 0;
  }
  try {
    const int n = (int)polar::unrolled_layouts(c->plan, c->llr_type).size();
    set(POLAR_OK);
    return n;
  } catch (const std::bad_alloc&) {
    set(POLAR_ENOMEM);
    return 0;
  }
}

polar_status polar_layout_info(const polar_code* c, int index, int* reg_stages, int* virtual_top,
                               int* wave_lds_bytes, int* virtual_mid) {
  if (!c || index < 0) return set(POLAR_EINVAL);
  try {
    const std::vector<polar::UnrolledLayout> all = polar::unrolled_layouts(c->plan, c->llr_type);
    if (index >= (int)all.size()) return set(POLAR_EINVAL);
    const polar::UnrolledLayout& L = all[(size_t)index];
    if (reg_stages) *reg_stages = L.nreg;
    if (virtual_top) *virtual_top = L.vtop;
    if (virtual_mid) *virtual_mid = L.vmid;
    if (wave_lds_bytes)
      *wave_lds_bytes = polar::wave_lds_bytes(c->plan.log2n, c->llr_type == POLAR_LLR_F32 ? 4 : 1, L.off_lds());
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  return set(POLAR_OK);
}

polar_status polar_set_layout(polar_code* c, int index) {
  if (!c) return set(POLAR_EINVAL);
  if (c->prepared) return set(POLAR_ESTATE);
  if (index < 0 || index >= polar_layout_count(c)) return set(POLAR_EINVAL);
  c->plan.layout = index;
  return set(POLAR_OK);
}

polar_status polar_set_kernel(polar_code* c, polar_kernel kernel) {
  if (!c) return set(POLAR_EINVAL);
  if (c->prepared) return set(POLAR_ESTATE);
  if (kernel != POLAR_KERNEL_SCHEDULE && kernel != POLAR_KERNEL_UNROLLED) return set(POLAR_EINVAL);
  c->kernel = kernel;
  return set(POLAR_OK);
}

polar_status polar_build_kernel(const polar_code* c) {
  if (!c) return set(POLAR_EINVAL);
  try {
    std::vector<char> code;
    std::string log;
    if (polar::unrolled_code_object(c->plan, c->llr_type, code, log) != 0) return set_msg(POLAR_ECOMPILE, log);
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  return set(POLAR_OK);
}

polar_status polar_prepare(polar_code* c) {
  if (!c) return set(POLAR_EINVAL);
  if (c->prepared) return set(POLAR_ESTATE);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set(POLAR_EDEVICE);
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return set(POLAR_EDEVICE);
  const int wave_bytes = polar::wave_lds_bytes(c->plan.log2n, c->llr_type == POLAR_LLR_F32 ? 4 : 1);
  if (wave_bytes > lds_max) return set(POLAR_ENOMEM);
  int wpb = lds_max / wave_bytes;
  if (wpb > 4) wpb = 4;
  if (wpb < 1) wpb = 1;
  if (c->kernel == POLAR_KERNEL_UNROLLED) {
    try {
      std::vector<char> code;
      std::string log;
      if (polar::unrolled_code_object(c->plan, c->llr_type, code, log) != 0) return set_msg(POLAR_ECOMPILE, log);
      if (polar::unrolled_load(code, c->unrolled) != 0) return set(POLAR_EDEVICE);
      c->unrolled.wave_bytes = polar::unrolled_wave_bytes(c->plan, c->llr_type);
      const int uw = lds_max / c->unrolled.wave_bytes;
      wpb = uw < 1 ? 1 : (uw > 4 ? 4 : uw);
    } catch (const std::bad_alloc&) {
      return set(POLAR_ENOMEM);
    }
  } else {
    if (polar::set_lds_limit(lds_max) != hipSuccess) return set(POLAR_EDEVICE);
    const size_t bytes = c->plan.dops.size() * sizeof(uint32_t);
    uint32_t* d = nullptr;
    if (polar::dev_malloc((void**)&d, bytes ? bytes : 4) != hipSuccess) return set(POLAR_ENOMEM);
    if (bytes && hipMemcpy(d, c->plan.dops.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      return set(POLAR_EDEVICE);
    }
    c->d_ops = d;
    c->nops = c->plan.nops;
  }
  c->device = dev;
  c->waves_per_block = wpb;
  c->prepared = true;
  return set(POLAR_OK);
}

void polar_destroy(polar_code* c) {
  if (!c) return;
  if (c->d_ops || c->unrolled.module) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != c->device) (void)hipSetDevice(c->device);
    if (c->d_ops) (void)hipFree(c->d_ops);
    polar::unrolled_unload(c->unrolled);
    if (cur != c->device) (void)hipSetDevice(cur);
  }
  delete c;
}

polar_status polar_last_status(void) { return g_last; }

polar_status polar_debug_fail_allocations(int after) {
  polar::arm_alloc_failure(after);
  return set(POLAR_OK);
}

const char* polar_last_message(void) { return g_message.c_str(); }

const char* polar_strerror(polar_status s) {
  switch (s) {
    case POLAR_OK: return "ok";
    case POLAR_EINVAL: return "invalid argument";
    case POLAR_ENOMEM: return "out of memory";
    case POLAR_EDEVICE: return "device error";
    case POLAR_ESTATE: return "invalid state";
    case POLAR_ECOMPILE: return "kernel compilation failed";
    case POLAR_EAGAIN: return "no room right now; poll and retry";
  }
  return "unknown status";
}

int polar_n(const polar_code* c) { return c ? c->plan.n : 0; }
int polar_k(const polar_code* c) { return c ? c->plan.k : 0; }

polar_status polar_frozen_mask(const polar_code* c, uint8_t* out) {
  if (!c || !out) return set(POLAR_EINVAL);
  std::memcpy(out, c->plan.frozen.data(), c->plan.n);
  return set(POLAR_OK);
}

polar_status polar_schedule(const polar_code* c, int32_t* kinds, int32_t* sizes, int32_t* offsets, int cap,
                            int* n_ops) {
  if (!c || cap < 0) return set(POLAR_EINVAL);
  const int total = (int)c->plan.lkind.size();
  for (int i = 0; i < total && i < cap; ++i) {
    if (kinds) kinds[i] = c->plan.lkind[i];
    if (sizes) sizes[i] = c->plan.lsize[i];
    if (offsets) offsets[i] = c->plan.loff[i];
  }
  if (n_ops) *n_ops = total;
  return set(POLAR_OK);
}

static_assert((int)POLAR_DOP_F == (int)polar::DOP_F && (int)POLAR_DOP_G_0R == (int)polar::DOP_G0R &&
                  (int)POLAR_DOP_COMBINE_R0 == (int)polar::DOP_CR0 && (int)POLAR_DOP_SPC == (int)polar::DOP_SPC &&
                  (int)POLAR_DOP_FLUSH == (int)polar::DOP_FLUSH && (int)POLAR_DOP_P01 == (int)polar::DOP_P01 &&
                  (int)POLAR_DOP_REPR1 == (int)polar::DOP_REPR1,
              "public device-op codes follow the kernels' codes");

polar_status polar_device_schedule(const polar_code* c, uint32_t* ops, int cap, int* n_ops) {
  if (!c || cap < 0) return set(POLAR_EINVAL);
  const int total = c->plan.nops;
  for (int i = 0; i < total && i < cap && ops; ++i) ops[i] = c->plan.dops[(size_t)i];
  if (n_ops) *n_ops = total;
  return set(POLAR_OK);
}

polar_status polar_encode(const polar_code* c, const uint8_t* info, int nframes, uint8_t* x) {
  if (!c || nframes < 0 || (nframes > 0 && (!info || !x))) return set(POLAR_EINVAL);
  const int n = c->plan.n, k = c->plan.k;
  const int in_row = (k + 7) / 8, out_row = (n + 7) / 8;
  const int words = (n + 63) / 64;
  std::vector<uint64_t> u(words);
  static const uint64_t kMask[6] = {0x5555555555555555ull, 0x3333333333333333ull, 0x0F0F0F0F0F0F0F0Full,
                                    0x00FF00FF00FF00FFull, 0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
  for (int fr = 0; fr < nframes; ++fr) {
    const uint8_t* in = info + (size_t)fr * in_row;
    std::fill(u.begin(), u.end(), 0ull);
    int j = 0;
    for (int i = 0; i < n; ++i) {
      if (c->plan.frozen[i]) continue;
      if ((in[j >> 3] >> (j & 7)) & 1) u[i >> 6] |= 1ull << (i & 63);
      ++j;
    }
    // x[i] ^= x[i+h] for every i with bit h clear: in-word levels, then word levels
    for (int l = 0, h = 1; h < 64 && h < n; ++l, h <<= 1)
      for (int w = 0; w < words; ++w) u[w] ^= (u[w] >> h) & kMask[l];
    for (int hw = 1; hw < words; hw <<= 1)
      for (int w = 0; w < words; ++w)
        if ((w & hw) == 0) u[w] ^= u[w + hw];
    uint8_t* out = x + (size_t)fr * out_row;
    for (int b = 0; b < out_row; ++b) out[b] = (uint8_t)(u[b >> 3] >> (8 * (b & 7)));
  }
  return set(POLAR_OK);
}

static polar_status decode_impl(const polar_code* c, const void* llr, int nframes, uint8_t* bits, void* trace,
                                void* stream) {
  if (!c || nframes < 0) return set(POLAR_EINVAL);
  if (!c->prepared) return set(POLAR_ESTATE);
  if (nframes == 0) return set(POLAR_OK);
  if (!llr || !bits) return set(POLAR_EINVAL);
  if (!llr_aligned(c->llr_type, llr)) return set(POLAR_EINVAL);
  if (c->llr_type == POLAR_LLR_F32 && trace && ((uintptr_t)trace & 3u) != 0) return set(POLAR_EINVAL);
  if (!on_device(c->device)) return set_msg(POLAR_ESTATE, "the current device is not the one the code was prepared on");
  const int rc = c->kernel == POLAR_KERNEL_UNROLLED
                     ? polar::unrolled_launch(c->unrolled, llr, nframes, bits, trace, c->waves_per_block, stream)
                     : polar::launch_decode(c->d_ops, c->nops, c->plan.log2n, c->plan.k, c->llr_type, llr, nframes,
                                            bits, trace, c->waves_per_block, stream);
  return set(rc == 0 ? POLAR_OK : POLAR_EDEVICE);
}

polar_status polar_decode(const polar_code* c, const void* llr, int nframes, uint8_t* bits, void* stream) {
  return decode_impl(c, llr, nframes, bits, nullptr, stream);
}

polar_status polar_decode_trace(const polar_code* c, const void* llr, int nframes, uint8_t* bits, void* trace,
                                void* stream) {
  if (nframes > 0 && !trace) return set(POLAR_EINVAL);
  return decode_impl(c, llr, nframes, bits, trace, stream);
}


polar_status polar_tune_layout(polar_code* c, const void* llr, int nframes, uint8_t* bits, void* stream,
                               int* chosen) {
  if (!c || nframes < 1 || !llr || !bits || !llr_aligned(c->llr_type, llr)) return set(POLAR_EINVAL);
  if (c->prepared || c->kernel != POLAR_KERNEL_UNROLLED) return set(POLAR_ESTATE);
  const int count = polar_layout_count(c);
  if (count < 1) return set(POLAR_ENOMEM);
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return set(POLAR_EDEVICE);
  // Every candidate's kernel is loaded at once and they are timed in rounds,
  // so that a clock still ramping up weighs on all of them alike: warm-up
  // rounds until 30 ms of decoding (at most 64 rounds), then 3 timed rounds
  // in which each layout runs a burst of 5 back-to-back launches (as in
  // use: one kernel again and again); each layout keeps its fastest burst.
  std::vector<polar::UnrolledKernel> ks;
  std::vector<int> wpb;
  std::vector<float> best_ms;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  polar_status st = POLAR_OK;
  std::string msg;
  try {
    ks.resize((size_t)count);
    wpb.resize((size_t)count);
    best_ms.assign((size_t)count, -1.0f);
    for (int i = 0; i < count && st == POLAR_OK; ++i) {
      c->plan.layout = i;
      std::vector<char> code;
      if (polar::unrolled_code_object(c->plan, c->llr_type, code, msg) != 0) {
        st = POLAR_ECOMPILE;
      } else if (polar::unrolled_load(code, ks[(size_t)i]) != 0) {
        st = POLAR_EDEVICE;
      } else {
        ks[(size_t)i].wave_bytes = polar::unrolled_wave_bytes(c->plan, c->llr_type);
        const int w = lds_max / ks[(size_t)i].wave_bytes;
        wpb[(size_t)i] = w < 1 ? 1 : (w > 4 ? 4 : w);
      }
    }
  } catch (const std::bad_alloc&) {
    st = POLAR_ENOMEM;
  }
  if (st == POLAR_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = POLAR_EDEVICE;
  float warm_ms = 0.0f;
  int warm_rounds = 0, timed_rounds = 0;
  while (st == POLAR_OK && timed_rounds < 3) {
    const bool timed = warm_ms >= 30.0f || warm_rounds >= 64;
    const int burst = timed ? 5 : 1;
    for (int i = 0; i < count && st == POLAR_OK; ++i) {
      if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) st = POLAR_EDEVICE;
      for (int b = 0; b < burst && st == POLAR_OK; ++b)
        if (polar::unrolled_launch(ks[(size_t)i], llr, nframes, bits, nullptr, wpb[(size_t)i], stream) != 0)
          st = POLAR_EDEVICE;
      if (st != POLAR_OK || hipEventRecord(e1, (hipStream_t)stream) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess) {
        st = POLAR_EDEVICE;
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= (float)burst;
      if (!timed)
        warm_ms += ms;
      else if (best_ms[(size_t)i] < 0.0f || ms < best_ms[(size_t)i])
        best_ms[(size_t)i] = ms;
    }
    if (timed)
      ++timed_rounds;
    else
      ++warm_rounds;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (polar::UnrolledKernel& k : ks) polar::unrolled_unload(k);
  int best = 0;
  for (int i = 1; i < count && st == POLAR_OK; ++i)
    if (best_ms[(size_t)i] < best_ms[(size_t)best]) best = i;
  if (st != POLAR_OK) {
    c->plan.layout = 0;
    return msg.empty() ? set(st) : set_msg(st, msg);
  }
  c->plan.layout = best;
  st = polar_prepare(c);
  if (st == POLAR_OK && chosen) *chosen = best;
  return st;
}

/* ------------------------------------------------------------------ batch */

}  // extern "C"

namespace {

int batch_occupancy(int wave_bytes, int lds_per_cu) {
  // waves of one SIMD (4 per CU) that the LDS allows, 1..4
  int per_cu = wave_bytes > 0 ? lds_per_cu / wave_bytes : 32;
  int w = per_cu / 4;
  return w < 1 ? 1 : (w > 4 ? 4 : w);
}

std::string batch_src(const polar_batch* b) {
  std::vector<const polar::Plan*> ps;
  for (const auto& p : b->plans) ps.push_back(&p);
  return polar::batch_source(ps, b->llr_type, b->waves_per_simd);
}

}  // namespace

extern "C" {

polar_batch* polar_batch_create(const polar_code* const* codes, int ncodes) {
  if (!codes || ncodes < 1 || ncodes > 255) {
    set(POLAR_EINVAL);
    return nullptr;
  }
  for (int i = 0; i < ncodes; ++i)
    if (!codes[i] || codes[i]->llr_type != codes[0]->llr_type) {
      set(POLAR_EINVAL);
      return nullptr;
    }
  polar_batch* b = polar::alloc_fails() ? nullptr : new (std::nothrow) polar_batch;
  if (!b) {
    set(POLAR_ENOMEM);
    return nullptr;
  }
  try {
    b->llr_type = codes[0]->llr_type;
    for (int i = 0; i < ncodes; ++i) {
      b->plans.push_back(codes[i]->plan);
      b->wave_bytes = std::max(b->wave_bytes, polar::unrolled_wave_bytes(codes[i]->plan, b->llr_type));
    }
  } catch (const std::bad_alloc&) {
    delete b;
    set(POLAR_ENOMEM);
    return nullptr;
  }
  b->waves_per_simd = batch_occupancy(b->wave_bytes, 160 * 1024);
  for (const polar::Plan& p : b->plans)  // and the register stages of every code's layout
    b->waves_per_simd = std::min(b->waves_per_simd, polar::unrolled_waves_per_simd(p, b->llr_type));
  set(POLAR_OK);
  return b;
}

polar_status polar_batch_build_kernel(const polar_batch* b) {
  if (!b) return set(POLAR_EINVAL);
  try {
    std::vector<char> code;
    std::string log;
    if (polar::source_code_object(batch_src(b), code, log) != 0) return set_msg(POLAR_ECOMPILE, log);
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  return set(POLAR_OK);
}

polar_status polar_batch_prepare(polar_batch* b) {
  if (!b) return set(POLAR_EINVAL);
  if (b->prepared) return set(POLAR_ESTATE);
  int dev = 0, cus = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return set(POLAR_EDEVICE);
  if (b->wave_bytes > lds_max) return set(POLAR_ENOMEM);
  try {
    std::vector<char> code;
    std::string log;
    if (polar::source_code_object(batch_src(b), code, log) != 0) return set_msg(POLAR_ECOMPILE, log);
    if (polar::batch_load(code, b->module, b->fn) != 0) return set(POLAR_EDEVICE);
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  b->device = dev;
  b->cus = cus;
  int wpb = lds_max / b->wave_bytes;
  b->waves_per_block = wpb < 1 ? 1 : (wpb > 4 ? 4 : wpb);
  // enough workgroups for every wave slot of the chip, each looping over frames
  b->blocks = cus * ((4 * b->waves_per_simd) / b->waves_per_block);
  if (b->blocks < 1) b->blocks = 1;
  b->prepared = true;
  return set(POLAR_OK);
}

polar_status polar_batch_set_frames(polar_batch* b, int nframes, const int32_t* code_index, const int64_t* llr_offset,
                                    const int64_t* bits_offset) {
  if (!b || nframes < 0 || (nframes > 0 && (!code_index || !llr_offset || !bits_offset))) return set(POLAR_EINVAL);
  if (!b->prepared) return set(POLAR_ESTATE);
  const int ncodes = (int)b->plans.size();
  std::vector<unsigned long long> desc;
  try {
    std::vector<int> order(nframes);
    for (int i = 0; i < nframes; ++i) {
      if (code_index[i] < 0 || code_index[i] >= ncodes || llr_offset[i] < 0 || bits_offset[i] < 0 ||
          bits_offset[i] >= (1ll << 56))
        return set(POLAR_EINVAL);
      order[i] = i;
    }
    // longest codes first, so the waves' strided walks finish together;
    // frames of one code next to each other, so neighbouring waves run the
    // same decoder (7% faster on a 15-code mix than by length alone)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      const int nx = b->plans[code_index[x]].n, ny = b->plans[code_index[y]].n;
      return nx != ny ? nx > ny : code_index[x] < code_index[y];
    });
    desc.resize(2 * (size_t)nframes);
    for (int j = 0; j < nframes; ++j) {
      const int i = order[j];
      desc[2 * j] = (unsigned long long)code_index[i] | ((unsigned long long)bits_offset[i] << 8);
      desc[2 * j + 1] = (unsigned long long)llr_offset[i];
    }
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  // decodes still running may read the old descriptors
  if (hipDeviceSynchronize() != hipSuccess) return set(POLAR_EDEVICE);
  if (nframes > b->desc_cap) {
    unsigned long long* d = nullptr;
    if (polar::dev_malloc((void**)&d, desc.size() * sizeof(unsigned long long)) != hipSuccess) return set(POLAR_ENOMEM);
    if (b->d_desc) (void)hipFree(b->d_desc);
    b->d_desc = d;
    b->desc_cap = nframes;
  }
  if (nframes > 0 &&
      hipMemcpy(b->d_desc, desc.data(), desc.size() * sizeof(unsigned long long), hipMemcpyHostToDevice) != hipSuccess)
    return set(POLAR_EDEVICE);
  b->nframes = nframes;
  return set(POLAR_OK);
}

polar_status polar_batch_decode_desc(const polar_batch* b, const uint64_t* desc, int nframes, const void* llr,
                                     uint8_t* bits, void* stream) {
  if (!b || nframes < 0) return set(POLAR_EINVAL);
  if (!b->prepared) return set(POLAR_ESTATE);
  if (nframes == 0) return set(POLAR_OK);
  if (!desc || !llr || !bits || !llr_aligned(b->llr_type, llr)) return set(POLAR_EINVAL);
  if (!on_device(b->device))
    return set_msg(POLAR_ESTATE, "the current device is not the one the batch was prepared on");
  const int rc = polar::batch_launch(b->fn, desc, nframes, llr, bits, b->wave_bytes, b->waves_per_block, b->blocks,
                                     stream);
  return set(rc == 0 ? POLAR_OK : POLAR_EDEVICE);
}

polar_status polar_batch_decode_frames_noalloc(const polar_batch* b, int nframes, const int32_t* code_index,
                                               const int64_t* llr_offset, const int64_t* bits_offset, const void* llr,
                                               uint8_t* bits, void* stream) {
  if (!b || nframes < 0) return set(POLAR_EINVAL);
  if (nframes > polar::kNoallocMaxFrames)
    return set_msg(POLAR_EINVAL, "polar_batch_decode_frames_noalloc takes at most 262144 frames per call");
  if (!b->prepared) return set(POLAR_ESTATE);
  if (nframes == 0) return set(POLAR_OK);
  if (!code_index || !llr_offset || !bits_offset || !llr || !bits || !llr_aligned(b->llr_type, llr))
    return set(POLAR_EINVAL);
  if (!on_device(b->device))
    return set_msg(POLAR_ESTATE, "the current device is not the one the batch was prepared on");
  void* desc = polar::noalloc_scratch(b->device);
  if (!desc) return set_msg(POLAR_EDEVICE, "no device address for the descriptor array");
  if (polar::noalloc_pack(desc, nframes, (int)b->plans.size(), code_index, llr_offset, bits_offset, stream) != 0)
    return set(POLAR_EDEVICE);
  const int rc = polar::batch_launch(b->fn, desc, nframes, llr, bits, b->wave_bytes, b->waves_per_block, b->blocks,
                                     stream);
  return set(rc == 0 ? POLAR_OK : POLAR_EDEVICE);
}

polar_status polar_batch_decode(const polar_batch* b, const void* llr, uint8_t* bits, void* stream) {
  if (!b) return set(POLAR_EINVAL);
  return polar_batch_decode_desc(b, (const uint64_t*)b->d_desc, b->nframes, llr, bits, stream);
}

polar_status polar_batch_tune(polar_batch* b, const void* llr, uint8_t* bits, void* stream) {
  if (!b) return set(POLAR_EINVAL);
  if (!b->prepared) return set(POLAR_ESTATE);
  if (b->nframes == 0) return set(POLAR_OK);
  if (!llr || !bits) return set(POLAR_EINVAL);
  if (!on_device(b->device))
    return set_msg(POLAR_ESTATE, "the current device is not the one the batch was prepared on");
  int lds_max = 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess)
    return set(POLAR_EDEVICE);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return set(POLAR_EDEVICE);
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set(POLAR_EDEVICE);
  }
  const int slots = b->cus * 4 * b->waves_per_simd;  // resident waves on the chip
  int best_wpb = b->waves_per_block, best_blocks = b->blocks;
  float best = -1.0f;
  polar_status st = POLAR_OK;
  for (int wpb = 1; wpb <= 4 && st == POLAR_OK; wpb <<= 1) {
    if (wpb * b->wave_bytes > lds_max) break;
    // resident grid, twice resident (late waves fill the tail), one wave per frame
    const int cands[3] = {slots / wpb, 2 * slots / wpb, (b->nframes + wpb - 1) / wpb};
    for (int c = 0; c < 3 && st == POLAR_OK; ++c) {
      const int blocks = cands[c] < 1 ? 1 : cands[c];
      float ms_best = -1.0f;
      for (int rep = 0; rep < 4; ++rep) {  // first launch warms up
        if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess ||
            polar::batch_launch(b->fn, b->d_desc, b->nframes, llr, bits, b->wave_bytes, wpb, blocks, stream) != 0 ||
            hipEventRecord(e1, (hipStream_t)stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          st = POLAR_EDEVICE;
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (ms_best < 0.0f || ms < ms_best)) ms_best = ms;
      }
      if (st == POLAR_OK && (best < 0.0f || ms_best < best)) {
        best = ms_best;
        best_wpb = wpb;
        best_blocks = blocks;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != POLAR_OK) return set(st);
  b->waves_per_block = best_wpb;
  b->blocks = best_blocks;
  return set(POLAR_OK);
}

polar_status polar_batch_launch_shape(const polar_batch* b, int* waves_per_block, int* blocks, int* wave_lds_bytes) {
  if (!b) return set(POLAR_EINVAL);
  if (waves_per_block) *waves_per_block = b->waves_per_block;
  if (blocks) *blocks = b->blocks;
  if (wave_lds_bytes) *wave_lds_bytes = b->wave_bytes;
  return set(POLAR_OK);
}

void polar_batch_destroy(polar_batch* b) {
  if (!b) return;
  if (b->module || b->d_desc) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != b->device) (void)hipSetDevice(b->device);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->module) (void)hipModuleUnload(b->module);
    if (cur != b->device) (void)hipSetDevice(cur);
  }
  delete b;
}

}  // extern "C"
