// Internal types shared by the host construction code, the C ABI and the
// HIP decode kernels of libpolar.  Not part of the public interface.
#pragma once
#include <stdint.h>

#include <vector>

#include "opcodes.h"

namespace polar {

// Decoder-tree node functions (the vocabulary of Listing 1) as they appear
// in the logical schedule returned by polar_schedule().
enum LogicalOp : int32_t {
  LOP_F = 0,      // eq. (1) into the left child
  LOP_G = 1,      // eq. (2) into the right child
  LOP_G0R = 2,    // eq. (2) with a Rate-0 left child (beta_l = 0)
  LOP_C = 3,      // eq. (3) combine
  LOP_C0R = 4,    // combine with a Rate-0 left child
  LOP_INFO = 5,   // Rate-1 leaf, eq. (4)
  LOP_REP = 6,    // repetition leaf (Sec. II-E)
  LOP_SPC = 7,    // single-parity-check leaf (Sec. II-E)
  LOP_CR0 = 8,    // combine with a Rate-0 right child (arbitrary masks only)
};

struct Plan {
  int n = 0;        // code length N
  int log2n = 0;
  int k = 0;        // information bits
  int algo = 0;     // 0 Fast-SSC, 1 SC
  int fuse = 1;     // Fast-SSC: fuse leaf-pair nodes of size <= 64 (DOP_P01 .. DOP_REPR1)
  int layout = 0;   // unrolled kernels: index into unrolled_layouts(), 0 = the default rule
  std::vector<uint8_t> frozen;          // N flags
  std::vector<int32_t> lkind, lsize, loff;  // logical schedule
  std::vector<uint32_t> dops;           // device schedule, one word per op, plus one padding op
  int nops = 0;
};

// Builds the logical and device schedules for plan.frozen / plan.algo.
void build_schedule(Plan& plan);

// Bhattacharyya-bound frozen set.  Returns false on bad arguments.
bool construct_frozen(int n, int k, double design_ebn0_db, std::vector<uint8_t>& frozen);

}  // namespace polar
