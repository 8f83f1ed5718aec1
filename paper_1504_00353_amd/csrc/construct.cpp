// Host-side code construction and decoder-schedule generation.
//
// Construction (Sec. II-A): the N-K least reliable bit channels are frozen.
// Reliability is the Bhattacharyya parameter z of the BPSK-AWGN channel at
// the design Eb/N0 (ln z0 = -R Eb/N0), pushed through the polarising kernel
// one level at a time: the first-decoded ("minus", f) channel of a pair gets
// 2z - z^2, the second ("plus", g) gets z^2.  Levels are built from the root
// split down, so the most significant index bit is the root split (natural
// indexing, Sec. II-A).  Everything is done on ln z in double precision
// since z underflows long before N = 32768.  Equal values are broken in
// favour of the higher index being an information bit.
//
// Schedule (Sec. II-B..E, Listing 1): a depth-first walk of the pruned
// decoder tree.  Fast-SSC stops at Rate-0, Rate-1, repetition and SPC nodes;
// plain SC decides single bits and only skips all-frozen sub-trees (their
// estimate is zero whatever the LLRs, so the decoded bits are unchanged).
// The device form is one 32-bit op per step of that walk.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "plan.h"

namespace polar {

bool construct_frozen(int n, int k, double design_ebn0_db, std::vector<uint8_t>& frozen) {
  if (n < 2 || n > kMaxN || (n & (n - 1)) || k < 1 || k > n) return false;
  const double es_n0 = (double)k / (double)n * std::pow(10.0, design_ebn0_db / 10.0);
  std::vector<double> lnz(1, -es_n0), next;
  while ((int)lnz.size() < n) {
    next.resize(lnz.size() * 2);
    for (size_t j = 0; j < lnz.size(); ++j) {
      const double L = lnz[j];
      next[2 * j] = L + std::log(2.0 - std::exp(L));  // minus channel: z -> 2z - z^2
      next[2 * j + 1] = 2.0 * L;                      // plus channel:  z -> z^2
    }
    lnz.swap(next);
  }
  std::vector<int> rank(n);
  std::iota(rank.begin(), rank.end(), 0);
  std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) {
    return lnz[a] < lnz[b] || (lnz[a] == lnz[b] && a > b);
  });
  frozen.assign(n, 1);
  for (int j = 0; j < k; ++j) frozen[rank[j]] = 0;
  return true;
}

namespace {

enum NodeKind { N_RATE0, N_RATE1, N_REP, N_SPC, N_INTERNAL };

struct Walker {
  Plan& p;
  std::vector<int> info_before;  // info_before[i] = # information bits at indices < i

  explicit Walker(Plan& plan) : p(plan) {
    info_before.assign(p.n + 1, 0);
    for (int i = 0; i < p.n; ++i) info_before[i + 1] = info_before[i] + (p.frozen[i] ? 0 : 1);
  }

  int frozen_count(int o, int size) const {
    // number of frozen indices in [o, o+size)
    return size - (info_before[o + size] - info_before[o]);
  }

  // Node kind for the device schedule.
  NodeKind device_kind(int o, int size) const {
    const int nf = frozen_count(o, size);
    if (nf == size) return N_RATE0;
    if (p.algo == 1) return size == 1 ? N_RATE1 : N_INTERNAL;
    if (nf == 0) return N_RATE1;
    if (size >= 2 && nf == size - 1 && !p.frozen[o + size - 1]) return N_REP;
    if (size >= 4 && nf == 1 && p.frozen[o]) return N_SPC;
    return N_INTERNAL;
  }

  // Node kind for the logical schedule: plain SC walks every node.
  NodeKind logical_kind(int o, int size) const {
    if (p.algo == 1 && size > 1) return N_INTERNAL;
    return device_kind(o, size);
  }

  void log(LogicalOp op, int size, int o) {
    p.lkind.push_back(op);
    p.lsize.push_back(size);
    p.loff.push_back(o);
  }

  void logical(int o, int stage) {
    const int size = 1 << stage;
    switch (logical_kind(o, size)) {
      case N_RATE0: return;
      case N_RATE1: log(LOP_INFO, size, o); return;
      case N_REP: log(LOP_REP, size, o); return;
      case N_SPC: log(LOP_SPC, size, o); return;
      case N_INTERNAL: break;
    }
    const int h = size / 2;
    const bool left_rate0 = p.algo == 0 && frozen_count(o, h) == h;
    if (left_rate0) {
      log(LOP_G0R, size, o);
      logical(o + h, stage - 1);
      log(LOP_C0R, size, o);
    } else {
      log(LOP_F, size, o);
      logical(o, stage - 1);
      log(LOP_G, size, o);
      logical(o + h, stage - 1);
      log(LOP_C, size, o);
    }
  }

  void dev(DeviceOp op, int stage, int o) { p.dops.push_back(pack_op(op, stage, o)); }

  // The fused op of an internal node at o whose children (size h) are a
  // Rate-0 or repetition node on the left and a Rate-1 or SPC node on the
  // right, else -1.
  int pair_op(int o, int h) const {
    const NodeKind l = device_kind(o, h), r = device_kind(o + h, h);
    if (l == N_RATE0 && r == N_RATE1) return DOP_P01;
    if (l == N_RATE0 && r == N_SPC) return DOP_0SPC;
    if (l == N_REP && r == N_SPC) return DOP_REPSPC;
    if (l == N_REP && r == N_RATE1) return DOP_REPR1;
    return -1;
  }

  // needed: some later G or combine reads this node's beta (the estimate of
  // the root and of the nodes on its right spine is never read).
  void device(int o, int stage, bool needed) {
    const int size = 1 << stage;
    const NodeKind kind = device_kind(o, size);
    switch (kind) {
      case N_RATE0: return;
      case N_RATE1: dev(DOP_R1, stage, o); break;
      case N_REP: dev(DOP_REP, stage, o); break;
      case N_SPC: dev(DOP_SPC, stage, o); break;
      case N_INTERNAL: {
        const int h = size / 2;
        const bool left_rate0 = frozen_count(o, h) == h;
        const bool right_rate0 = frozen_count(o + h, h) == h;
        const int pair = p.algo == 0 && p.fuse && stage <= kRegStages ? pair_op(o, h) : -1;
        if (pair >= 0) {
          dev((DeviceOp)pair, stage, o);
        } else if (left_rate0) {
          dev(DOP_G0R, stage, o);
          device(o + h, stage - 1, needed);
          if (needed) dev(DOP_C0R, stage, o);
        } else if (right_rate0) {
          dev(DOP_F, stage, o);
          device(o, stage - 1, true);
          if (needed) dev(DOP_CR0, stage, o);
        } else {
          dev(DOP_F, stage, o);
          device(o, stage - 1, true);
          dev(DOP_G, stage, o);
          device(o + h, stage - 1, needed);
          if (needed) dev(DOP_C, stage, o);
        }
        break;
      }
    }
    // A finished size-64 node hands its estimate to a parent that keeps beta in LDS.
    if (needed && stage == kRegStages && p.log2n > kRegStages) dev(DOP_FLUSH, stage, o);
  }
};

}  // namespace

void build_schedule(Plan& plan) {
  plan.lkind.clear();
  plan.lsize.clear();
  plan.loff.clear();
  plan.dops.clear();
  Walker w(plan);
  w.logical(0, plan.log2n);
  w.device(0, plan.log2n, false);
  plan.nops = (int)plan.dops.size();
  plan.dops.push_back(pack_op(DOP_END, 0, 0));  // the kernel prefetches one op ahead
}

}  // namespace polar
