// Generated per-code (unrolled) decode kernels: source generation, the
// on-disk code object cache, module loading and launch.
#pragma once
#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "plan.h"

namespace polar {

struct UnrolledKernel {
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
  hipFunction_t fn_trace = nullptr;
  int wave_bytes = 0;  // LDS slot of one wavefront
};

// How a generated kernel places the widest alpha stages: nreg stages in
// registers, with vtop the stage below the root not stored at all, and with
// vmid (float, N = 32768) not the stage below the register stage either.
struct UnrolledLayout {
  int nreg = 0;
  int vtop = 0;
  int vmid = 0;
  // top stages that are not in LDS
  int off_lds() const { return nreg + vtop + vmid; }
};
// The layout the plan's kernel uses: candidate p.layout of
// unrolled_layouts() (0, the default rule, when out of range).
UnrolledLayout unrolled_layout(const Plan& p, int llr_type);
// Every layout the decoder templates accept for this plan, the default rule
// first; the autotuner times them.
std::vector<UnrolledLayout> unrolled_layouts(const Plan& p, int llr_type);
// LDS bytes of one wavefront of the generated kernel of this plan.
int unrolled_wave_bytes(const Plan& p, int llr_type);
// VGPRs of a layout's register stages.
int unrolled_stage_vgprs(const Plan& p, int llr_type, UnrolledLayout L);
// VGPRs the int8 decoders need besides their register stages.
constexpr int kRegWorkingSet = 56;
// Waves per SIMD the plan's generated kernel is compiled for (its register
// budget): what its LDS slot allows and, for int8, what its register stages
// leave room for.  1..4.
int unrolled_waves_per_simd(const Plan& p, int llr_type);

// HIP source of the two kernels (plain and tracing) for the plan's device
// schedule and the LLR type (0 int8, 1 float).
std::string unrolled_source(const Plan& p, int llr_type);

// Code object of the plan's kernels from the cache, or compiled now and
// stored.  0 on success; -1 with the compiler log otherwise.
int unrolled_code_object(const Plan& p, int llr_type, std::vector<char>& code, std::string& log);

// Code object for any generated source (cache, else compile and store).
int source_code_object(const std::string& src, std::vector<char>& code, std::string& log);

// HIP source of the persistent batch kernel over several codes of one LLR
// type; waves_per_simd: the occupancy its register use is held to.
std::string batch_source(const std::vector<const Plan*>& plans, int llr_type, int waves_per_simd);
int batch_load(const std::vector<char>& code, hipModule_t& module, hipFunction_t& fn);
int batch_launch(hipFunction_t fn, const void* desc, int nframes, const void* llr, uint8_t* bits, int wave_bytes,
                 int waves_per_block, int blocks, void* stream);

// Loads a code object on the current device.  0 on success.
int unrolled_load(const std::vector<char>& code, UnrolledKernel& k);
void unrolled_unload(UnrolledKernel& k);

// Launches the loaded kernel; returns the hipError_t of the launch.
int unrolled_launch(const UnrolledKernel& k, const void* llr, int nframes, uint8_t* bits, void* trace,
                    int waves_per_block, void* stream);

}  // namespace polar
