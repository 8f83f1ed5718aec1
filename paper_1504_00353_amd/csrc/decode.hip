// Fast-SSC / SC polar decoding kernels for gfx950 (MI355X).
//
// One wavefront decodes one frame by walking the device schedule built on
// the host (a depth-first pre-order of the pruned decoder tree, Listing 1
// form).  The schedule is wave-uniform, so every branch below is a scalar
// branch and the 64 lanes work on the elements of the current node.
//
// Storage of the LLR messages alpha (per-stage buffers, Sec. III-B.3):
//   * stages 0..6 (node sizes 1..64) live in VGPRs, element i in lane i;
//     f and g pull the partner element i + N_v/2 with a lane shuffle;
//   * stages 7..log2(N)-1 live in LDS, one buffer per stage;
//   * stage log2(N) is the channel frame, read straight from global memory.
// Bit estimates beta use one N-bit array updated in place (Sec. III-B.2):
// nodes of size <= 64 keep their bits in a 64-bit wave-uniform window (so
// combines are scalar ALU work and g picks its sign from the window), and a
// finished size-64 node flushes the window to the LDS bit array that larger
// nodes use.  Leaves emit their information bits directly: for a node
// covering bits [o, o+N_v), u[o..o+N_v) = beta_v G_{N_v} (the polar transform
// is its own inverse), so no final re-encode of the whole frame is needed.
//
// Arithmetic: int8 LLRs are processed as 32-bit integers with the 8-bit
// semantics of Listing 4 (g saturates to [-127, 127]); float LLRs use one
// IEEE round-to-nearest add per g and the halving-tree order for the
// repetition sum, so results are bit-identical to a sequential decoder that
// follows the same definitions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace polar {
namespace {

template <typename T>
struct Arith;

template <>
struct Arith<int8_t> {
  typedef int R;  // register value
  typedef int S;  // repetition sum (exact)
  static __device__ __forceinline__ R chan(int8_t v) { return v < -127 ? -127 : (int)v; }
  static __device__ __forceinline__ R from(int8_t v) { return (int)v; }
  static __device__ __forceinline__ int8_t to(R v) { return (int8_t)v; }
  // eq. (1): sgn(a)sgn(b)min(|a|,|b|) == max(min(a,b), -max(a,b))
  static __device__ __forceinline__ R f(R a, R b) { return max(min(a, b), -max(a, b)); }
  static __device__ __forceinline__ R g(R a, R b, bool beta) {
    R r = beta ? b - a : b + a;
    return min(max(r, -127), 127);
  }
  static __device__ __forceinline__ R g0(R a, R b) { return min(max(b + a, -127), 127); }
  static __device__ __forceinline__ bool neg(R v) { return v < 0; }
  static __device__ __forceinline__ R mag(R v) { return v < 0 ? -v : v; }
  static __device__ __forceinline__ S add(S a, S b) { return a + b; }
  static __device__ __forceinline__ R mn(R a, R b) { return min(a, b); }
  static constexpr int kBig = 1 << 20;
};

template <>
struct Arith<float> {
  typedef float R;
  typedef float S;
  static __device__ __forceinline__ R chan(float v) { return v; }
  static __device__ __forceinline__ R from(float v) { return v; }
  static __device__ __forceinline__ float to(R v) { return v; }
  static __device__ __forceinline__ R f(R a, R b) { return fmaxf(fminf(a, b), -fmaxf(a, b)); }
  static __device__ __forceinline__ R g(R a, R b, bool beta) {
    return beta ? __fsub_rn(b, a) : __fadd_rn(b, a);
  }
  static __device__ __forceinline__ R g0(R a, R b) { return __fadd_rn(b, a); }
  static __device__ __forceinline__ bool neg(R v) { return v < 0.0f; }
  static __device__ __forceinline__ R mag(R v) { return fabsf(v); }
  static __device__ __forceinline__ S add(S a, S b) { return __fadd_rn(a, b); }
  static __device__ __forceinline__ R mn(R a, R b) { return fminf(a, b); }
  static constexpr float kBig = 3.0e38f;
};

// Orders the wave's LDS traffic across lanes and keeps the compiler from
// moving memory operations over op boundaries.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t low_mask(int bits) {
  return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
}

// u = x G_n on up to 64 bits (x[i] ^= x[i+h] for i with bit h clear).
__device__ __forceinline__ uint64_t transform64(uint64_t x, int size) {
  if (size > 1) x ^= (x >> 1) & 0x5555555555555555ull;
  if (size > 2) x ^= (x >> 2) & 0x3333333333333333ull;
  if (size > 4) x ^= (x >> 4) & 0x0F0F0F0F0F0F0F0Full;
  if (size > 8) x ^= (x >> 8) & 0x00FF00FF00FF00FFull;
  if (size > 16) x ^= (x >> 16) & 0x0000FFFF0000FFFFull;
  if (size > 32) x ^= (x >> 32) & 0x00000000FFFFFFFFull;
  return x;
}

__device__ __forceinline__ uint32_t transform32(uint32_t x) {
  x ^= (x >> 1) & 0x55555555u;
  x ^= (x >> 2) & 0x33333333u;
  x ^= (x >> 4) & 0x0F0F0F0Fu;
  x ^= (x >> 8) & 0x00FF00FFu;
  x ^= (x >> 16) & 0x0000FFFFu;
  return x;
}

// OR `nbits` (<= 64) bits of val into the LDS bit row at bit position pos.
__device__ __forceinline__ void put_bits(uint32_t* out, uint32_t pos, uint64_t val, int lane) {
  const uint32_t w = pos >> 5, sh = pos & 31;
  uint32_t part;
  if (lane == 0)
    part = (uint32_t)(val << sh);
  else if (lane == 1)
    part = sh ? (uint32_t)(val >> (32 - sh)) : (uint32_t)(val >> 32);
  else
    part = sh ? (uint32_t)(val >> (64 - sh)) : 0u;
  if (lane < 3 && part) out[w + lane] |= part;
}

template <typename T>
struct Wave {
  typedef Arith<T> A;
  typedef typename A::R R;

  int lane;
  int log2n;
  const T* ch;        // channel frame (global)
  T* alpha;           // LDS: stage s (7 <= s < log2n) at alpha + 2^s - 128
  uint32_t* beta;     // LDS: N bits
  uint32_t* out;      // LDS: K bits
  T* tr;              // global trace row or null
  R a[kRegStages + 1];
  uint64_t win;       // beta bits of the current 64-aligned block

  __device__ __forceinline__ T* stage(int s) const { return alpha + ((1 << s) - 128); }

  __device__ __forceinline__ R load_in(int s, int i) const {
    return s == log2n ? A::chan(ch[i]) : A::from(stage(s)[i]);
  }

  __device__ __forceinline__ bool beta_bit(int i) const { return (beta[i >> 5] >> (i & 31)) & 1u; }

  // ---------------- nodes of size <= 64: registers, shuffles, ballots ----
  template <int K>
  __device__ __forceinline__ void small_fg(uint32_t code, int o) {
    constexpr int H = 1 << (K - 1);
    const R x = a[K];
    const R y = __shfl_down(x, H, 64);
    if (code == DOP_F) {
      a[K - 1] = A::f(x, y);
    } else if (code == DOP_G) {
      const bool b = (win >> ((o + lane) & 63)) & 1ull;  // beta_l[lane], o = node offset mod 64
      a[K - 1] = A::g(x, y, b);
    } else {
      a[K - 1] = A::g0(x, y);
    }
  }

  template <int K>
  __device__ __forceinline__ void small_leaf(uint32_t code, int o, uint32_t outpos) {
    constexpr int NV = 1 << K;
    const int off = o & 63;
    const uint64_t m = low_mask(NV);
    const R x = a[K];
    if (tr && lane < NV) tr[o + lane] = A::to(x);
    uint64_t hd = (uint64_t)__ballot(A::neg(x)) & m;
    if (code == DOP_R1) {
      win = (win & ~(m << off)) | (hd << off);
      put_bits(out, outpos, transform64(hd, NV), lane);
    } else if (code == DOP_REP) {
      typename A::S s = x;
#pragma unroll
      for (int h = NV / 2; h >= 1; h >>= 1) s = A::add(s, __shfl_down(s, h, 64));
      const bool bit = __shfl(s, 0, 64) < 0;
      win = (win & ~(m << off)) | ((bit ? m : 0ull) << off);
      put_bits(out, outpos, bit ? 1ull : 0ull, lane);
    } else {  // DOP_SPC
      if (__popcll(hd) & 1) {
        R v = lane < NV ? A::mag(x) : (R)A::kBig;
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) v = A::mn(v, __shfl_xor(v, h, 64));
        const uint64_t cand = (uint64_t)__ballot(lane < NV && A::mag(x) == v);
        hd ^= 1ull << (__ffsll((unsigned long long)cand) - 1);
      }
      win = (win & ~(m << off)) | (hd << off);
      put_bits(out, outpos, transform64(hd, NV) >> 1, lane);
    }
  }

  __device__ __forceinline__ void small_combine(uint32_t code, int k, int o) {
    const int h = 1 << (k - 1);
    const int off = o & 63;
    const uint64_t m = low_mask(h);
    const uint64_t r = (win >> (off + h)) & m;
    if (code == DOP_C)
      win ^= r << off;
    else if (code == DOP_C0R)
      win = (win & ~(m << off)) | (r << off);
    else  // DOP_CR0
      win &= ~(m << (off + h));
  }

  // ---------------- nodes of size >= 128: LDS stages ---------------------
  __device__ __forceinline__ void big_fg(uint32_t code, int k, int o) {
    const int h = 1 << (k - 1);
    if (k == kRegStages + 1) {  // output is register stage 6
      const R x = load_in(k, lane), y = load_in(k, lane + h);
      if (code == DOP_F)
        a[kRegStages] = A::f(x, y);
      else if (code == DOP_G)
        a[kRegStages] = A::g(x, y, beta_bit(o + lane));
      else
        a[kRegStages] = A::g0(x, y);
      return;
    }
    T* dst = stage(k - 1);
    for (int i = lane; i < h; i += 64) {
      const R x = load_in(k, i), y = load_in(k, i + h);
      R r;
      if (code == DOP_F)
        r = A::f(x, y);
      else if (code == DOP_G)
        r = A::g(x, y, beta_bit(o + i));
      else
        r = A::g0(x, y);
      dst[i] = A::to(r);
    }
  }

  __device__ __forceinline__ void big_combine(uint32_t code, int k, int o) {
    const int h = 1 << (k - 1);
    const int words = h >> 5;
    uint32_t* l = beta + (o >> 5);
    uint32_t* r = beta + ((o + h) >> 5);
    for (int j = lane; j < words; j += 64) {
      if (code == DOP_C)
        l[j] ^= r[j];
      else if (code == DOP_C0R)
        l[j] = r[j];
      else
        r[j] = 0u;
    }
  }

  // Information bits of a big Rate-1 or SPC leaf: u = beta G over the
  // leaf's W words, word j held by lane j % 64 in register j / 64.
  template <int K>
  __device__ __forceinline__ void big_emit(const uint32_t* src, uint32_t outpos, bool spc) {
    constexpr int W = (1 << K) / 32;
    constexpr int D = W > 64 ? W / 64 : 1;
    constexpr int L = W > 64 ? 64 : W;
    uint32_t v[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int j = t * 64 + lane;
      v[t] = (lane < L) ? transform32(src[j]) : 0u;
    }
#pragma unroll
    for (int dw = 1; dw < L; dw <<= 1) {
#pragma unroll
      for (int t = 0; t < D; ++t) {
        const uint32_t other = __shfl_down(v[t], dw, 64);
        if ((lane & dw) == 0) v[t] ^= other;
      }
    }
#pragma unroll
    for (int dt = 1; dt < D; dt <<= 1) {
#pragma unroll
      for (int t = 0; t < D; ++t)
        if ((t & dt) == 0) v[t] ^= v[t + dt];
    }
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int j = t * 64 + lane;
      if (lane >= L) continue;
      uint32_t word = v[t];
      uint32_t pos = outpos + 32u * j;
      if (spc) {
        if (j == 0) {
          word >>= 1;  // u_0 is the frozen bit of the SPC node
        } else {
          pos -= 1;
        }
      }
      const uint32_t w = pos >> 5, sh = pos & 31;
      const uint32_t lo = word << sh;
      const uint32_t hi = sh ? (word >> (32 - sh)) : 0u;
      if (lo) atomicOr(&out[w], lo);
      if (hi) atomicOr(&out[w + 1], hi);
    }
  }

  __device__ __forceinline__ void emit_dispatch(int k, const uint32_t* src, uint32_t outpos, bool spc) {
    switch (k) {
      case 7: big_emit<7>(src, outpos, spc); break;
      case 8: big_emit<8>(src, outpos, spc); break;
      case 9: big_emit<9>(src, outpos, spc); break;
      case 10: big_emit<10>(src, outpos, spc); break;
      case 11: big_emit<11>(src, outpos, spc); break;
      case 12: big_emit<12>(src, outpos, spc); break;
      case 13: big_emit<13>(src, outpos, spc); break;
      case 14: big_emit<14>(src, outpos, spc); break;
      default: big_emit<15>(src, outpos, spc); break;
    }
  }

  __device__ __forceinline__ void big_leaf(uint32_t code, int k, int o, uint32_t outpos) {
    const int nv = 1 << k;
    const int words = nv >> 5;
    uint32_t* bw = beta + (o >> 5);
    if (code == DOP_REP) {
      typename A::S s;
      if (tr)
        for (int i = lane; i < nv; i += 64) tr[o + i] = A::to(load_in(k, i));
      if constexpr (sizeof(T) == 1) {
        // exact integer sum: the order is free
        typename A::S acc = 0;
        for (int i = lane; i < nv; i += 64) acc = A::add(acc, load_in(k, i));
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) acc = A::add(acc, __shfl_xor(acc, h, 64));
        s = acc;
      } else {
        // halving tree s_i <- s_i + s_{i+m/2}: the top levels in the (dead)
        // LDS buffers of the stages below this leaf, the last 64 in lanes
        int m = nv;
        int src_stage = k;
        while (m / 2 > 64) {
          const int h = m / 2;
          int dst_stage = 31 - __clz(h);
          T* dst = stage(dst_stage);
          for (int i = lane; i < h; i += 64)
            dst[i] = A::to(A::add(load_in(src_stage, i), load_in(src_stage, i + h)));
          wave_sync();
          src_stage = dst_stage;
          m = h;
        }
        typename A::S acc = A::add(load_in(src_stage, lane), load_in(src_stage, lane + 64));
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) acc = A::add(acc, __shfl_down(acc, h, 64));
        s = __shfl(acc, 0, 64);
      }
      const bool bit = s < 0;
      for (int j = lane; j < words; j += 64) bw[j] = bit ? ~0u : 0u;
      if (lane == 0 && bit) out[outpos >> 5] |= 1u << (outpos & 31);
      return;
    }
    // Rate-1 and SPC: hard decisions, one 32-bit word of beta per lane
    int parity = 0;
    R best = (R)A::kBig;
    int best_i = 0x7fffffff;
    for (int j = lane; j < words; j += 64) {
      uint32_t d = 0;
      for (int b = 0; b < 32; ++b) {
        const int i = 32 * j + b;
        const R x = load_in(k, i);
        if (tr) tr[o + i] = A::to(x);
        d |= (uint32_t)A::neg(x) << b;
        const R mg = A::mag(x);
        if (mg < best) {
          best = mg;
          best_i = i;
        }
      }
      bw[j] = d;
      parity ^= __popc(d) & 1;
    }
    if (code == DOP_SPC) {
      const uint64_t odd = (uint64_t)__ballot(parity != 0);
      if (__popcll(odd) & 1) {
        R v = best;
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) v = A::mn(v, __shfl_xor(v, h, 64));
        int idx = (best == v) ? best_i : 0x7fffffff;
#pragma unroll
        for (int h = 32; h >= 1; h >>= 1) idx = min(idx, __shfl_xor(idx, h, 64));
        wave_sync();
        if (lane == 0) bw[idx >> 5] ^= 1u << (idx & 31);
      }
    }
    wave_sync();
    emit_dispatch(k, bw, outpos, code == DOP_SPC);
  }

  __device__ __forceinline__ void small_dispatch(uint32_t code, int k, int o, uint32_t outpos) {
    if (code <= DOP_G0R) {
      switch (k) {
        case 1: small_fg<1>(code, o); break;
        case 2: small_fg<2>(code, o); break;
        case 3: small_fg<3>(code, o); break;
        case 4: small_fg<4>(code, o); break;
        case 5: small_fg<5>(code, o); break;
        default: small_fg<6>(code, o); break;
      }
    } else if (code <= DOP_CR0) {
      small_combine(code, k, o);
    } else if (code == DOP_FLUSH) {
      if (lane < 2) beta[(o >> 5) + lane] = (uint32_t)(win >> (32 * lane));
    } else {
      switch (k) {
        case 0: small_leaf<0>(code, o, outpos); break;
        case 1: small_leaf<1>(code, o, outpos); break;
        case 2: small_leaf<2>(code, o, outpos); break;
        case 3: small_leaf<3>(code, o, outpos); break;
        case 4: small_leaf<4>(code, o, outpos); break;
        case 5: small_leaf<5>(code, o, outpos); break;
        default: small_leaf<6>(code, o, outpos); break;
      }
    }
  }

  __device__ __forceinline__ void load_small_root(int n) {
    const R x = lane < n ? A::chan(ch[lane]) : (R)0;
    switch (log2n) {
      case 1: a[1] = x; break;
      case 2: a[2] = x; break;
      case 3: a[3] = x; break;
      case 4: a[4] = x; break;
      case 5: a[5] = x; break;
      default: a[6] = x; break;
    }
  }
};

}  // namespace

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// LDS bytes one wave needs for a code: alpha stages 7..log2n-1, the N-bit
// beta array (when N > 64) and the K-bit output row.
int wave_lds_bytes(int log2n, int k, int llr_type) {
  const int elem = llr_type == 1 ? 4 : 1;
  const int n = 1 << log2n;
  const int alpha = log2n > 7 ? (n - 128) * elem : 0;
  const int beta = log2n > kRegStages ? n / 8 : 0;
  const int out = ((k + 31) / 32) * 4;
  return align16(alpha) + align16(beta) + align16(out);
}

template <typename T>
__global__ void __launch_bounds__(256) decode_kernel(const uint32_t* __restrict__ ops, int nops, int log2n,
                                                     int kbits, const T* __restrict__ llr, int nframes,
                                                     uint8_t* __restrict__ bits, T* __restrict__ trace,
                                                     int wave_bytes) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int frame = blockIdx.x * (blockDim.x >> 6) + wid;
  if (frame >= nframes) return;  // wave-uniform; no block-level barriers follow

  const int n = 1 << log2n;
  const int elem = (int)sizeof(T);
  unsigned char* base = smem + (size_t)wid * wave_bytes;
  const int alpha_bytes = log2n > 7 ? (n - 128) * elem : 0;
  const int beta_bytes = log2n > kRegStages ? n / 8 : 0;
  const int out_words = (kbits + 31) / 32;

  Wave<T> w;
  w.lane = lane;
  w.log2n = log2n;
  w.ch = llr + (size_t)frame * n;
  w.alpha = (T*)base;
  w.beta = (uint32_t*)(base + align16(alpha_bytes));
  w.out = (uint32_t*)(base + align16(alpha_bytes) + align16(beta_bytes));
  w.tr = trace ? trace + (size_t)frame * n : nullptr;
  w.win = 0;
#pragma unroll
  for (int s = 0; s <= kRegStages; ++s) w.a[s] = 0;

  for (int j = lane; j < out_words; j += 64) w.out[j] = 0u;
  if (log2n <= kRegStages) w.load_small_root(n);
  wave_sync();

  for (int pc = 0; pc < nops; ++pc) {
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(ops[2 * pc]);
    const uint32_t w1 = __builtin_amdgcn_readfirstlane(ops[2 * pc + 1]);
    const uint32_t code = w0 & 0xffu;
    const int k = (int)((w0 >> 8) & 0xffu);
    const int o = (int)(w0 >> 16);
    if (k <= kRegStages) {
      w.small_dispatch(code, k, o, w1);
    } else if (code <= DOP_G0R) {
      w.big_fg(code, k, o);
    } else if (code <= DOP_CR0) {
      w.big_combine(code, k, o);
    } else {
      w.big_leaf(code, k, o, w1);
    }
    wave_sync();
  }

  const int row = (kbits + 7) / 8;
  const unsigned char* ob = (const unsigned char*)w.out;
  uint8_t* dst = bits + (size_t)frame * row;
  for (int b = lane; b < row; b += 64) dst[b] = ob[b];
}

int launch_decode(const uint32_t* ops, int nops, int log2n, int kbits, int llr_type, const void* llr,
                  int nframes, uint8_t* bits, void* trace, int waves_per_block, void* stream) {
  const int wave_bytes = wave_lds_bytes(log2n, kbits, llr_type);
  const int blocks = (nframes + waves_per_block - 1) / waves_per_block;
  const dim3 grid(blocks), block(64 * waves_per_block);
  const size_t lds = (size_t)wave_bytes * waves_per_block;
  hipStream_t s = (hipStream_t)stream;
  if (llr_type == 1) {
    hipLaunchKernelGGL(decode_kernel<float>, grid, block, lds, s, ops, nops, log2n, kbits, (const float*)llr,
                       nframes, bits, (float*)trace, wave_bytes);
  } else {
    hipLaunchKernelGGL(decode_kernel<int8_t>, grid, block, lds, s, ops, nops, log2n, kbits, (const int8_t*)llr,
                       nframes, bits, (int8_t*)trace, wave_bytes);
  }
  return (int)hipGetLastError();
}

int set_lds_limit(int llr_type, int bytes) {
  hipError_t e;
  if (llr_type == 1)
    e = hipFuncSetAttribute((const void*)decode_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  else
    e = hipFuncSetAttribute((const void*)decode_kernel<int8_t>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return (int)e;
}

}  // namespace polar
