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
