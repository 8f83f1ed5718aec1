// Allocation-free batch decode: the frame-descriptor queue that the batch
// kernel walks lives in a fixed device array of this library instead of
// memory that polar_batch_set_frames() allocates.  For callers that cannot
// allocate device memory (code under HIP graph capture, tight serving
// loops).
//
// One array per device, shared by every call on that device and kept until
// the process ends; calls that overlap on one device race on it.  Host code
// reaches the array only through the address hipGetSymbolAddress() returns
// for the current device (the array's name in host code is a host-side
// stand-in, not a device address).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "noalloc.h"

namespace polar {

namespace {

// Two 64-bit words per frame, the batch kernel's descriptor format.
static __device__ __align__(256) unsigned long long scratch[2 * kNoallocMaxFrames];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};

// desc[2i] = code | bits offset << 8, desc[2i+1] = LLR offset.  A frame with
// a code index outside [0, ncodes), a negative offset or a bits offset of
// 2^56 or more gets code 255, which the batch kernel skips.
__global__ void __launch_bounds__(256) pack_descriptors(unsigned long long* __restrict__ desc, int nframes,
                                                        int ncodes, const int32_t* __restrict__ code_index,
                                                        const int64_t* __restrict__ llr_offset,
                                                        const int64_t* __restrict__ bits_offset) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nframes) return;
  const int32_t c = code_index[i];
  const int64_t lo = llr_offset[i], bo = bits_offset[i];
  const bool ok = c >= 0 && c < ncodes && lo >= 0 && bo >= 0 && bo < (1ll << 56);
  desc[2 * i] = ok ? ((unsigned long long)c | ((unsigned long long)bo << 8)) : 255ull;
  desc[2 * i + 1] = ok ? (unsigned long long)lo : 0ull;
}

}  // namespace

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[device]) {
    // once per device, with that device current (the caller's check)
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[device] = p;
  }
  return g_ptr[device];
}

int noalloc_pack(void* desc, int nframes, int ncodes, const int32_t* code_index, const int64_t* llr_offset,
                 const int64_t* bits_offset, void* stream) {
  const int threads = 256;
  const int blocks = (nframes + threads - 1) / threads;
  void* args[] = {&desc, &nframes, &ncodes, (void*)&code_index, (void*)&llr_offset, (void*)&bits_offset};
  return (int)hipLaunchKernel((const void*)pack_descriptors, dim3(blocks), dim3(threads), args, 0,
                              (hipStream_t)stream);
}

}  // namespace polar
