// Device op codes of the decoder schedule, shared by the host schedule
// builder, the schedule-interpreting kernel and the generated per-code
// kernels.  Plain C++ with no includes so that the run-time compiler can
// take it as is.
#pragma once

namespace polar {

// One op is one 32-bit word:  code | stage << 8 | node_offset << 16.
// "stage" is log2 of the node size Nv; F/G/G0R read stage k and write
// stage k-1; leaves and combines act on a node of stage k.  Decision nodes
// append their information bits to the output in schedule order, which is
// increasing index order.
enum DeviceOp : unsigned {
  DOP_F = 0,      // eq. (1) into the left child
  DOP_G = 1,      // eq. (2) into the right child
  DOP_G0R = 2,    // eq. (2) with a Rate-0 left child (beta_l = 0)
  DOP_C = 3,      // eq. (3) combine
  DOP_C0R = 4,    // combine with a Rate-0 left child (copy)
  DOP_CR0 = 5,    // combine with a Rate-0 right child (clear the right half)
  DOP_R1 = 6,     // Rate-1 leaf, eq. (4)
  DOP_REP = 7,    // repetition leaf (Sec. II-E)
  DOP_SPC = 8,    // single-parity-check leaf (Sec. II-E)
  DOP_FLUSH = 9,  // write the 64-bit beta window of a finished size-64 node to LDS
  DOP_END = 10,   // padding after the last op
  // Fused nodes of size <= 64 whose two children are leaves (the P_01, 0SPC
  // and RepSPC functions of the Fast-SSC library, Sec. II-E, and Rep-R1):
  // the whole subtree f / leaf / g / leaf / combine in one op, with the
  // arithmetic of the separate ops.
  DOP_P01 = 11,     // left Rate-0, right Rate-1
  DOP_0SPC = 12,    // left Rate-0, right SPC
  DOP_REPSPC = 13,  // left repetition, right SPC
  DOP_REPR1 = 14,   // left repetition, right Rate-1
};

constexpr bool is_pair_op(unsigned code) { return code >= DOP_P01 && code <= DOP_REPR1; }

constexpr int kRegStages = 6;  // stages 0..6 (sizes 1..64) are register resident
constexpr int kMaxLog2N = 15;  // N <= 32768
constexpr int kMaxN = 1 << kMaxLog2N;

constexpr unsigned pack_op(unsigned code, int stage, int offset) {
  return code | ((unsigned)stage << 8) | ((unsigned)offset << 16);
}

// LDS bytes one wavefront needs: a 128-byte g sign table, the alpha stages
// 7..log2n-1-nreg (elem bytes per LLR; the top nreg stages may live in
// registers instead) and the N-bit beta array, each 16-byte aligned.
constexpr int alpha_lds_bytes(int log2n, int elem, int nreg) {
  return log2n - nreg > 7 ? ((1 << (log2n - nreg)) - 128) * elem : 0;
}
constexpr int wave_lds_bytes(int log2n, int elem, int nreg = 0) {
  return 128 + ((alpha_lds_bytes(log2n, elem, nreg) + 15) & ~15) + (((log2n > 6 ? (1 << log2n) / 8 : 0) + 15) & ~15);
}

}  // namespace polar
