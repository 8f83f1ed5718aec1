// The allocation-free batch decode's fixed descriptor array (noalloc.hip).
#pragma once
#include <stdint.h>

namespace polar {

// Frames one allocation-free batch call can take (16 bytes each: 4 MiB of
// device memory per device, held until the process ends).
constexpr int kNoallocMaxFrames = 262144;

// Device address of the descriptor array on `device`, which must be the
// current device; looked up on the first call per device.  Null on error.
void* noalloc_scratch(int device);

// Writes the batch kernel's descriptors for nframes frames (device arrays)
// into desc on the stream; returns the launch's hipError_t.
int noalloc_pack(void* desc, int nframes, int ncodes, const int32_t* code_index, const int64_t* llr_offset,
                 const int64_t* bits_offset, void* stream);

}  // namespace polar
