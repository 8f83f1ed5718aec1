// Library-internal definitions of the opaque C ABI objects, shared by the
// C ABI (api.cpp) and the request server (server.cpp).
#pragma once
#include <hip/hip_runtime_api.h>

#include <vector>

#include "../../include/polar.h"
#include "plan.h"
#include "unrolled.h"

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

struct polar_batch {
  std::vector<polar::Plan> plans;  // copies of the codes' schedules
  int llr_type = POLAR_LLR_I8;
  int wave_bytes = 0;              // LDS slot of one wave: the largest code's need
  int waves_per_simd = 1;          // occupancy the generated kernel's registers are held to
  bool prepared = false;
  int device = -1;
  int cus = 0;
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
  int waves_per_block = 4;
  int blocks = 0;
  unsigned long long* d_desc = nullptr;  // descriptors from polar_batch_set_frames
  int desc_cap = 0;
  int nframes = 0;
};

// Records a status for polar_last_status() and returns it.
polar_status polar_set_status(polar_status s);

namespace polar {
// Every allocation the library makes (its objects, device memory, pinned
// host memory) asks this first; true when polar_debug_fail_allocations()
// has armed a failure for this allocation.
bool alloc_fails();
void arm_alloc_failure(int after);
// hipMalloc / hipHostMalloc through the allocation-failure hook.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t pinned_malloc(void** p, size_t bytes);
}  // namespace polar
