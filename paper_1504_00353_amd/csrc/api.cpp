// C ABI of libpolar: argument validation, status codes, code objects,
// device upload and the host encoder.  See include/polar.h.
#include <hip/hip_runtime_api.h>

#include <cstring>
#include <string>
#include <new>
#include <vector>

#include "../../include/polar.h"
#include "plan.h"
#include "unrolled.h"

namespace polar {
int launch_decode(const uint32_t* ops, int nops, int log2n, int kbits, int llr_type, const void* llr, int nframes,
                  uint8_t* bits, void* trace, int waves_per_block, void* stream);
int set_lds_limit(int llr_type, int bytes);
}  // namespace polar

struct polar_code {
  polar::Plan plan;
  int llr_type = POLAR_LLR_I8;
  int kernel = POLAR_KERNEL_SCHEDULE;
  bool prepared = false;
  int device = -1;
  uint32_t* d_ops = nullptr;
  int nops = 0;
  int waves_per_block = 1;
  polar::UnrolledKernel unrolled;
};

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

int log2_exact(int n) {
  if (n < 2 || n > polar::kMaxN || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

polar_code* make_code(int n, std::vector<uint8_t>&& frozen) {
  polar_code* c = new (std::nothrow) polar_code;
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

}  // namespace

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

polar_status polar_configure(polar_code* c, int algo, int llr_type) {
  if (!c) return set(POLAR_EINVAL);
  if (c->prepared) return set(POLAR_ESTATE);
  if ((algo != POLAR_ALGO_FASTSSC && algo != POLAR_ALGO_SC) || (llr_type != POLAR_LLR_I8 && llr_type != POLAR_LLR_F32))
    return set(POLAR_EINVAL);
  try {
    c->plan.algo = algo;
    c->llr_type = llr_type;
    polar::build_schedule(c->plan);
  } catch (const std::bad_alloc&) {
    return set(POLAR_ENOMEM);
  }
  return set(POLAR_OK);
}

polar_status polar_set_kernel(polar_code* c, int kernel) {
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
    } catch (const std::bad_alloc&) {
      return set(POLAR_ENOMEM);
    }
  } else {
    if (polar::set_lds_limit(c->llr_type, wpb * wave_bytes) != hipSuccess) return set(POLAR_EDEVICE);
    const size_t bytes = c->plan.dops.size() * sizeof(uint32_t);
    uint32_t* d = nullptr;
    if (hipMalloc((void**)&d, bytes ? bytes : 4) != hipSuccess) return set(POLAR_ENOMEM);
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

const char* polar_last_message(void) { return g_message.c_str(); }

const char* polar_strerror(polar_status s) {
  switch (s) {
    case POLAR_OK: return "ok";
    case POLAR_EINVAL: return "invalid argument";
    case POLAR_ENOMEM: return "out of memory";
    case POLAR_EDEVICE: return "device error";
    case POLAR_ESTATE: return "invalid state";
    case POLAR_ECOMPILE: return "kernel compilation failed";
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
  if (((uintptr_t)llr & 3u) != 0) return set(POLAR_EINVAL);
  if (c->llr_type == POLAR_LLR_F32 && trace && ((uintptr_t)trace & 3u) != 0) return set(POLAR_EINVAL);
  const int rc = c->kernel == POLAR_KERNEL_UNROLLED
                     ? polar::unrolled_launch(c->unrolled, c->plan.log2n, c->llr_type, llr, nframes, bits, trace,
                                              c->waves_per_block, stream)
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

}  // extern "C"
