// Internal types shared by the host construction code, the C ABI and the
// HIP decode kernels of libpolar.  Not part of the public interface.
#pragma once
#include <stdint.h>

#include <vector>

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

// Device op codes.  One op is one 32-bit word:
//   code | stage << 8 | node_offset << 16      (node_offset < 2^16)
// "stage" is log2 of the node size Nv; F/G/G0R read stage k and write
// stage k-1; leaves and combines act on a node of stage k.  Decision nodes
// append their information bits to the output in schedule order, which is
// increasing index order.
enum DeviceOp : uint32_t {
  DOP_F = 0,
  DOP_G = 1,
  DOP_G0R = 2,
  DOP_C = 3,
  DOP_C0R = 4,
  DOP_CR0 = 5,
  DOP_R1 = 6,
  DOP_REP = 7,
  DOP_SPC = 8,
  DOP_FLUSH = 9,  // write the 64-bit beta window of a finished size-64 node to LDS
  DOP_END = 10,   // padding after the last op
};

constexpr int kRegStages = 6;       // stages 0..6 (sizes 1..64) are register resident
constexpr int kMaxLog2N = 15;       // N <= 32768
constexpr int kMaxN = 1 << kMaxLog2N;

inline uint32_t pack_op(uint32_t code, int stage, int offset) {
  return code | ((uint32_t)stage << 8) | ((uint32_t)offset << 16);
}

struct Plan {
  int n = 0;        // code length N
  int log2n = 0;
  int k = 0;        // information bits
  int algo = 0;     // 0 Fast-SSC, 1 SC
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
