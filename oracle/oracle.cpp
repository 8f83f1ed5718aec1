// Plain, slow, CPU reference of SC and Fast-SSC polar decoding.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
// includes this file; only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark load it.  It shares no header, table or
// helper with the GPU library: every step is written out again here, in the
// order and notation of Giard et al., "Low-Latency Software Polar Decoders"
// (Sec. II), so a reader can check it against the paper by eye.
//
// Arithmetic domains (the decoder is a template over them):
//   double  -- reference precision;
//   float   -- IEEE binary32, one rounding per add (built -ffp-contract=off);
//   I8Sat   -- 8-bit saturating fixed point (Sec. III-A.1, Listing 4):
//              values in [-127, 127]; only g can grow a magnitude and it
//              saturates symmetrically.
//
// Readings taken where the paper is silent (each is also listed in the
// design notes of the repository):
//   * hard decision HD(x) = 1 iff x < 0, so HD(+0) = HD(-0) = 0 (eq. (4),
//     and the repetition rule of Sec. II-E: ">= 0 -> 0");
//   * repetition sum: the halving tree s_i <- s_i + s_{i+m/2}, m = Nv..2,
//     which is exactly the G_0R cascade plain SC would run; int8 sums are
//     exact (32-bit, no saturation);
//   * SPC: the flipped bit is the LOWEST index attaining min |alpha|
//     (Listing 2 finds the first matching lane);
//   * node precedence Rate-0, Rate-1, repetition (Nv >= 2), SPC (Nv >= 4);
//   * int8 channel value -128 is read as -127 (symmetric range);
//   * construction: Bhattacharyya bound in the log domain, ties between
//     equally reliable indices favour the higher index as information bit.
//
// Parity pins live in tests/test_oracle_*.py.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Arithmetic domains
// ---------------------------------------------------------------------------

// 8-bit saturating fixed point.  Storage int8, partial sums int32.
struct I8Sat {
  typedef int8_t value;
  typedef int32_t sum;
  static value channel(value x) { return x < -127 ? (value)-127 : x; }
  // eq. (1): sgn(a) sgn(b) min(|a|, |b|); exact in 8 bits.
  static value f(value a, value b) {
    int ma = a < 0 ? -(int)a : (int)a;
    int mb = b < 0 ? -(int)b : (int)b;
    int m = ma < mb ? ma : mb;
    bool negative = (a < 0) != (b < 0);
    return (value)(negative ? -m : m);
  }
  // eq. (2) with a saturating adder clamped to [-127, 127] (Listing 4).
  static value g(value a, value b, int beta) {
    int r = beta ? (int)b - (int)a : (int)b + (int)a;
    if (r > 127) r = 127;
    if (r < -127) r = -127;
    return (value)r;
  }
  static sum to_sum(value x) { return (sum)x; }
  static sum add(sum s, sum t) { return s + t; }
  static bool hd(value x) { return x < 0; }
  static bool sum_negative(sum s) { return s < 0; }
  static int magnitude(value x) { return x < 0 ? -(int)x : (int)x; }
};

// IEEE binary32 or binary64.
template <typename T>
struct Real {
  typedef T value;
  typedef T sum;
  static value channel(value x) { return x; }
  static value f(value a, value b) {
    T ma = std::fabs(a), mb = std::fabs(b);
    T m = ma < mb ? ma : mb;
    bool negative = (a < 0) != (b < 0);
    return negative ? -m : m;
  }
  static value g(value a, value b, int beta) { return beta ? b - a : b + a; }
  static sum to_sum(value x) { return x; }
  static sum add(sum s, sum t) { return s + t; }
  static bool hd(value x) { return x < 0; }
  static bool sum_negative(sum s) { return s < 0; }
  static T magnitude(value x) { return std::fabs(x); }
};

// ---------------------------------------------------------------------------
// Constituent-code classification (Sec. II-D and II-E)
// ---------------------------------------------------------------------------
enum Kind { RATE0 = 0, RATE1 = 1, REP = 2, SPC = 3, INTERNAL = 4 };

Kind classify(const uint8_t* frozen, int n, bool fast_ssc) {
  if (!fast_ssc && n > 1) return INTERNAL;  // plain SC decides single bits only
  int nfrozen = 0;
  for (int i = 0; i < n; ++i) nfrozen += frozen[i] ? 1 : 0;
  if (nfrozen == n) return RATE0;
  if (nfrozen == 0) return RATE1;
  if (n >= 2 && nfrozen == n - 1 && !frozen[n - 1]) return REP;
  if (n >= 4 && nfrozen == 1 && frozen[0]) return SPC;
  return INTERNAL;
}

// Op log entries, named after the functions of Listing 1.
enum LogOp { L_F = 0, L_G = 1, L_G0R = 2, L_C = 3, L_C0R = 4, L_INFO = 5, L_REP = 6, L_SPC = 7 };

// ---------------------------------------------------------------------------
// The decoder: a direct depth-first recursion over the decoder tree.
// ---------------------------------------------------------------------------
template <typename A>
struct Decoder {
  typedef typename A::value V;
  typedef typename A::sum S;

  const uint8_t* frozen;  // N flags, natural index order
  bool fast_ssc;
  V* trace;               // N entries or null: alpha_v of every non-Rate-0 leaf
  std::vector<int>* log_kind;
  std::vector<int>* log_size;

  void log(int kind, int size) {
    if (log_kind) {
      log_kind->push_back(kind);
      log_size->push_back(size);
    }
  }

  // Decode the node whose bits are u[o .. o+n) given alpha (n values);
  // returns beta (n bits) = the node's codeword estimate.
  std::vector<uint8_t> node(const std::vector<V>& alpha, int o, int n) {
    std::vector<uint8_t> beta(n, 0);
    Kind kind = classify(frozen + o, n, fast_ssc);
    if (kind == RATE0) {
      // Sec. II-D: a frozen sub-tree outputs the zero vector.
      return beta;
    }
    if (kind != INTERNAL && trace) {
      for (int i = 0; i < n; ++i) trace[o + i] = alpha[i];
    }
    if (kind == RATE1) {
      // Sec. II-D / eq. (4): element-wise threshold detection.
      log(L_INFO, n);
      for (int i = 0; i < n; ++i) beta[i] = A::hd(alpha[i]) ? 1 : 0;
      return beta;
    }
    if (kind == REP) {
      // Sec. II-E, repetition code: sum the LLRs, threshold, replicate.
      log(L_REP, n);
      std::vector<S> s(n);
      for (int i = 0; i < n; ++i) s[i] = A::to_sum(alpha[i]);
      for (int m = n; m >= 2; m /= 2)
        for (int i = 0; i < m / 2; ++i) s[i] = A::add(s[i], s[i + m / 2]);
      uint8_t bit = A::sum_negative(s[0]) ? 1 : 0;
      for (int i = 0; i < n; ++i) beta[i] = bit;
      return beta;
    }
    if (kind == SPC) {
      // Sec. II-E, single-parity-check code: hard decisions, parity, and
      // if the parity is odd flip the least reliable bit.
      log(L_SPC, n);
      int parity = 0;
      for (int i = 0; i < n; ++i) {
        beta[i] = A::hd(alpha[i]) ? 1 : 0;
        parity ^= beta[i];
      }
      if (parity) {
        int j = 0;
        for (int i = 1; i < n; ++i)
          if (A::magnitude(alpha[i]) < A::magnitude(alpha[j])) j = i;  // lowest index wins ties
        beta[j] ^= 1;
      }
      return beta;
    }
    // Internal node: left child first, then right child (Sec. II-C).
    int h = n / 2;
    std::vector<uint8_t> beta_l, beta_r;
    std::vector<V> child(h);
    bool left_rate0 = fast_ssc_left_rate0(o, h);
    if (left_rate0) {
      // Listing 1: G_0R then Combine_0R when the left child is Rate-0.
      log(L_G0R, n);
      for (int i = 0; i < h; ++i) child[i] = A::g(alpha[i], alpha[i + h], 0);
      beta_l.assign(h, 0);
      beta_r = node(child, o + h, h);
      log(L_C0R, n);
    } else {
      log(L_F, n);
      for (int i = 0; i < h; ++i) child[i] = A::f(alpha[i], alpha[i + h]);  // eq. (1)
      beta_l = node(child, o, h);
      log(L_G, n);
      for (int i = 0; i < h; ++i) child[i] = A::g(alpha[i], alpha[i + h], beta_l[i]);  // eq. (2)
      beta_r = node(child, o + h, h);
      log(L_C, n);
    }
    for (int i = 0; i < h; ++i) {  // eq. (3)
      beta[i] = beta_l[i] ^ beta_r[i];
      beta[i + h] = beta_r[i];
    }
    return beta;
  }

  // The Rate-0 shortcut for a left child is the SSC/Fast-SSC pruning; plain
  // SC walks every node down to single bits.
  bool fast_ssc_left_rate0(int o, int h) {
    if (!fast_ssc) return false;
    for (int i = 0; i < h; ++i)
      if (!frozen[o + i]) return false;
    return true;
  }
};

// x = u F^{(x)n}: for h = 1, 2, 4, .., N/2: x[i] ^= x[i+h] for i with bit h clear
// (Sec. II-A; G_4 is printed there).  The transform is its own inverse.
void polar_transform(int n, uint8_t* x) {
  for (int h = 1; h < n; h *= 2)
    for (int i = 0; i < n; ++i)
      if ((i & h) == 0) x[i] ^= x[i + h];
}

bool is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

template <typename A>
int decode_frames(int n, const uint8_t* frozen, int algo, int nframes,
                  const typename A::value* llr, uint8_t* u_out, uint8_t* x_out,
                  typename A::value* trace, int nthreads) {
  typedef typename A::value V;
  if (!is_pow2(n) || n < 2 || nframes < 0 || !frozen || (!llr && nframes > 0)) return 1;
  if (nthreads < 1) nthreads = 1;
  auto work = [&](int first, int last) {
    for (int fr = first; fr < last; ++fr) {
      Decoder<A> d;
      d.frozen = frozen;
      d.fast_ssc = (algo == 0);
      d.trace = trace ? trace + (size_t)fr * n : nullptr;
      d.log_kind = nullptr;
      d.log_size = nullptr;
      if (d.trace)
        for (int i = 0; i < n; ++i) d.trace[i] = (V)0;
      std::vector<V> alpha(n);
      for (int i = 0; i < n; ++i) alpha[i] = A::channel(llr[(size_t)fr * n + i]);
      std::vector<uint8_t> beta = d.node(alpha, 0, n);
      // C9: x_hat = beta_root; u_hat = x_hat F^{(x)n}.
      if (x_out) std::memcpy(x_out + (size_t)fr * n, beta.data(), n);
      polar_transform(n, beta.data());
      if (u_out) std::memcpy(u_out + (size_t)fr * n, beta.data(), n);
    }
  };
  if (nthreads == 1 || nframes < 2) {
    work(0, nframes);
  } else {
    std::vector<std::thread> pool;
    int per = (nframes + nthreads - 1) / nthreads;
    for (int t = 0; t < nthreads; ++t) {
      int a = t * per, b = std::min(nframes, a + per);
      if (a < b) pool.emplace_back(work, a, b);
    }
    for (auto& th : pool) th.join();
  }
  return 0;
}

}  // namespace

extern "C" {

// Code construction (Sec. II-A): freeze the N-K least reliable bit channels.
// Reliability = Bhattacharyya parameter z of the BPSK-AWGN channel at the
// design Eb/N0, propagated through the kernel: the "minus" channel (left
// child, f) gets z -> 2z - z^2 and the "plus" channel (right child, g) gets
// z -> z^2.  The first (most significant) index bit is the root split.
// Computed in the log domain: ln z0 = -R Eb/N0, then L -> L + ln(2 - e^L) or
// L -> 2L.  oracle_bhattacharyya gives ln z of every index for a given ln z0
// (for the BEC with erasure probability e, ln z0 = ln e and the recursion is
// exact).  Returns 0 on success.
int oracle_bhattacharyya(int n, double lnz0, double* lnz) {
  if (!is_pow2(n) || n < 2 || !lnz) return 1;
  int levels = 0;
  while ((1 << levels) < n) ++levels;
  for (int i = 0; i < n; ++i) {
    double L = lnz0;
    for (int b = levels - 1; b >= 0; --b) {
      if ((i >> b) & 1)
        L = 2.0 * L;
      else
        L = L + std::log(2.0 - std::exp(L));
    }
    lnz[i] = L;
  }
  return 0;
}

// ln z of every bit channel of an (n, k) code designed at Eb/N0 = design_ebn0_db
// (the reliabilities oracle_construct ranks): BPSK over AWGN at the design
// point has Es/N0 = R Eb/N0 with R = k/n, and its Bhattacharyya parameter is
// z0 = exp(-Es/N0).  *lnz0 (may be null) receives ln z0.  Returns 0 on success.
int oracle_construct_lnz(int n, int k, double design_ebn0_db, double* lnz, double* lnz0) {
  if (!is_pow2(n) || n < 2 || k < 0 || k > n || !lnz) return 1;
  double rate = (double)k / (double)n;
  double es_n0 = rate * std::pow(10.0, design_ebn0_db / 10.0);
  if (lnz0) *lnz0 = -es_n0;
  return oracle_bhattacharyya(n, -es_n0, lnz);
}

int oracle_construct(int n, int k, double design_ebn0_db, uint8_t* frozen) {
  if (!is_pow2(n) || n < 2 || k < 0 || k > n || !frozen) return 1;
  std::vector<double> lnz(n);
  oracle_construct_lnz(n, k, design_ebn0_db, lnz.data(), nullptr);
  // Rank: most reliable (smallest ln z) first; equal values -> higher index first.
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    if (lnz[a] != lnz[b]) return lnz[a] < lnz[b];
    return a > b;
  });
  for (int i = 0; i < n; ++i) frozen[i] = 1;
  for (int j = 0; j < k; ++j) frozen[order[j]] = 0;
  return 0;
}

// Encoder: x = u G_N with u given one bit per byte (frozen entries must be 0).
int oracle_encode(int n, int nframes, const uint8_t* u, uint8_t* x) {
  if (!is_pow2(n) || nframes < 0) return 1;
  for (int fr = 0; fr < nframes; ++fr) {
    std::memcpy(x + (size_t)fr * n, u + (size_t)fr * n, n);
    polar_transform(n, x + (size_t)fr * n);
  }
  return 0;
}

// Decoders.  algo 0 = Fast-SSC, 1 = plain SC.  Outputs (each optional):
// u_out / x_out: nframes*N bytes of 0/1; trace: nframes*N values, alpha_v of
// every non-Rate-0 leaf written at the leaf's own index range, 0 elsewhere.
int oracle_decode_i8(int n, const uint8_t* frozen, int algo, int nframes, const int8_t* llr,
                     uint8_t* u_out, uint8_t* x_out, int8_t* trace, int nthreads) {
  return decode_frames<I8Sat>(n, frozen, algo, nframes, llr, u_out, x_out, trace, nthreads);
}
int oracle_decode_f32(int n, const uint8_t* frozen, int algo, int nframes, const float* llr,
                      uint8_t* u_out, uint8_t* x_out, float* trace, int nthreads) {
  return decode_frames<Real<float>>(n, frozen, algo, nframes, llr, u_out, x_out, trace, nthreads);
}
int oracle_decode_f64(int n, const uint8_t* frozen, int algo, int nframes, const double* llr,
                      uint8_t* u_out, uint8_t* x_out, double* trace, int nthreads) {
  return decode_frames<Real<double>>(n, frozen, algo, nframes, llr, u_out, x_out, trace, nthreads);
}

// The sequence of node functions one decode runs (Listing 1 vocabulary):
// kinds 0 F, 1 G, 2 G_0R, 3 Combine, 4 Combine_0R, 5 Info, 6 Repetition, 7 SPC.
// Returns the number of entries (may exceed cap; only cap are written).
int oracle_schedule(int n, const uint8_t* frozen, int algo, int* kinds, int* sizes, int cap) {
  if (!is_pow2(n) || n < 2) return -1;
  std::vector<int> lk, ls;
  Decoder<Real<double>> d;
  d.frozen = frozen;
  d.fast_ssc = (algo == 0);
  d.trace = nullptr;
  d.log_kind = &lk;
  d.log_size = &ls;
  std::vector<double> alpha(n, 1.0);
  d.node(alpha, 0, n);
  for (int i = 0; i < (int)lk.size() && i < cap; ++i) {
    kinds[i] = lk[i];
    sizes[i] = ls[i];
  }
  return (int)lk.size();
}

// Single constituent-code decoders, for the brute-force ML pins.
// kind: 1 Rate-1, 2 repetition, 3 SPC.  beta: n bytes.
int oracle_node_i8(int kind, int n, const int8_t* alpha, uint8_t* beta) {
  std::vector<uint8_t> fz(n, 0);
  if (kind == REP) { for (int i = 0; i < n - 1; ++i) fz[i] = 1; }
  else if (kind == SPC) fz[0] = 1;
  else if (kind != RATE1) return 1;
  if (classify(fz.data(), n, true) != kind) return 1;
  Decoder<I8Sat> d;
  d.frozen = fz.data(); d.fast_ssc = true; d.trace = nullptr; d.log_kind = nullptr; d.log_size = nullptr;
  std::vector<int8_t> a(alpha, alpha + n);
  std::vector<uint8_t> b = d.node(a, 0, n);
  std::memcpy(beta, b.data(), n);
  return 0;
}
int oracle_node_f64(int kind, int n, const double* alpha, uint8_t* beta) {
  std::vector<uint8_t> fz(n, 0);
  if (kind == REP) { for (int i = 0; i < n - 1; ++i) fz[i] = 1; }
  else if (kind == SPC) fz[0] = 1;
  else if (kind != RATE1) return 1;
  if (classify(fz.data(), n, true) != kind) return 1;
  Decoder<Real<double>> d;
  d.frozen = fz.data(); d.fast_ssc = true; d.trace = nullptr; d.log_kind = nullptr; d.log_size = nullptr;
  std::vector<double> a(alpha, alpha + n);
  std::vector<uint8_t> b = d.node(a, 0, n);
  std::memcpy(beta, b.data(), n);
  return 0;
}

// The two message updates, exposed for the kernel-level pins.
int oracle_f_i8(int a, int b) { return I8Sat::f((int8_t)a, (int8_t)b); }
int oracle_g_i8(int a, int b, int beta) { return I8Sat::g((int8_t)a, (int8_t)b, beta); }
double oracle_f_f64(double a, double b) { return Real<double>::f(a, b); }
double oracle_g_f64(double a, double b, int beta) { return Real<double>::g(a, b, beta); }

}  // extern "C"
