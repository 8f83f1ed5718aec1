// Schedule-interpreting Fast-SSC / SC decode kernel for gfx950: one
// wavefront per frame runs the code's device schedule, read from memory at
// run time, so one kernel serves every code.  The op implementations are in
// decode_ops.h.
#include "decode_ops.h"

namespace polar {

template <class P>
__global__ void __launch_bounds__(256) decode_kernel(const uint32_t* __restrict__ ops, int nops, int log2n,
                                                     int kbits, const typename P::Chan* __restrict__ llr,
                                                     int nframes, uint8_t* __restrict__ bits,
                                                     typename P::Chan* __restrict__ trace, int wave_bytes) {
  extern __shared__ __align__(16) uint32_t smem[];
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; readfirstlane keeps frame pointers scalar
  const int wid = (int)rfl(threadIdx.x >> 6);
  const int frame = blockIdx.x * (blockDim.x >> 6) + wid;
  if (frame >= nframes) return;  // no block-level barriers follow

  Dec<P> d;
  d.init((LDS unsigned char*)smem + wid * wave_bytes, lane, log2n, kbits, llr, frame, bits, trace);

  // The schedule is read 64 ops at a time, one op per lane, with the next
  // block in flight; each op is taken out of the block with readlane.  The
  // block is moved into place by an opaque copy at the block boundary, so
  // the wait for its load happens there and not at every op.
  const __amdgpu_buffer_rsrc_t opr = __builtin_amdgcn_make_buffer_rsrc((void*)ops, 0, nops * 4, 0x00020000);
  uint32_t nxt = __builtin_amdgcn_raw_buffer_load_b32(opr, 4 * lane, 0, 0);
  for (int pb = 0; pb < nops; pb += 64) {
    uint32_t blk;
    asm volatile("v_mov_b32 %0, %1" : "=v"(blk) : "v"(nxt));
    nxt = __builtin_amdgcn_raw_buffer_load_b32(opr, 4 * (pb + 64 + lane), 0, 0);
    const int cnt = (int)rfl((uint32_t)min(64, nops - pb));
    for (int j = 0; j < cnt; ++j) d.step((uint32_t)__builtin_amdgcn_readlane((int)blk, j));
  }
  d.finish();
}

int launch_decode(const uint32_t* ops, int nops, int log2n, int kbits, int llr_type, const void* llr, int nframes,
                  uint8_t* bits, void* trace, int waves_per_block, void* stream) {
  int wb = wave_lds_bytes(log2n, llr_type == 1 ? 4 : 1);
  const dim3 grid((nframes + waves_per_block - 1) / waves_per_block), block(64 * waves_per_block);
  const size_t lds = (size_t)wb * waves_per_block;
  // the launch's own status: an error left on the thread by an earlier,
  // unrelated call is neither reported nor cleared here
  void* args[] = {(void*)&ops, (void*)&nops, (void*)&log2n, (void*)&kbits, (void*)&llr,
                  (void*)&nframes, (void*)&bits, (void*)&trace, (void*)&wb};
  const void* fn = llr_type == 1 ? (const void*)decode_kernel<PF32> : (const void*)decode_kernel<PI8>;
  return (int)hipLaunchKernel(fn, grid, block, args, lds, (hipStream_t)stream);
}

// Allows the schedule kernels every dynamic LDS size the device offers, so
// a launch never depends on which code was prepared last.
int set_lds_limit(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)decode_kernel<PF32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)decode_kernel<PI8>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return (int)e;
}

}  // namespace polar
