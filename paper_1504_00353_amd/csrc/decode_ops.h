// Fast-SSC / SC polar decoder ops for gfx950 (MI355X): the device code shared
// by the schedule-interpreting kernel and the generated per-code kernels.
//
// One wavefront decodes one frame by running the device schedule built on
// the host: the ops of a depth-first pre-order walk of the pruned decoder
// tree (the form of Listing 1).  The schedule is the same for every frame of
// a code, so every branch is wave-uniform.  The schedule is either read at
// run time (decode.hip) or compiled into a kernel of its own with every op
// argument a constant (the generated kernels; the paper's unrolled decoder).
//
// This header is also handed to the run-time compiler, so it includes
// nothing when compiled that way.
//
// Where the LLR messages alpha live (one buffer per stage, Sec. III-B.3):
//   stages 0..6  (node sizes 1..64): one element per lane, f32 VGPRs.  f and
//                g fetch the partner element i + N_v/2 with DPP row shifts
//                or the gfx950 permlane16/32 swaps;
//   stages 7..   LDS, natural order, int8 (int8 codes) or f32.  A lane works
//                on 16 contiguous bytes (or 4 for small nodes), so the pair
//                i, i + N_v/2 of f and g is lane-local; int8 values are
//                computed as packed 16-bit integers scaled by 256;
//   stage log2N  the channel frame, read with bounds-checked buffer loads.
// Bit estimates beta use one in-place N-bit array (Sec. III-B.2): nodes of
// size <= 64 keep their 64-bit block in a wave-uniform register (combines
// are scalar ALU work, g turns the bits into a lane predicate); a finished
// size-64 node flushes it to the LDS bit array used by larger nodes.
// Output: for a node covering bits [o, o+N_v), u[o..o+N_v) = beta_v G_{N_v}
// (the transform is its own inverse), so each decision node appends its
// information bits, in index order, to a 64-bit scalar accumulator that is
// stored 8 bytes at a time.
//
// Arithmetic: int8 LLRs follow Listing 4 (g saturates to [-127, 127]);
// float LLRs use one IEEE add per g and the halving-tree repetition sum, so
// both are bit-identical to a sequential decoder with the same definitions.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
typedef signed char int8_t;
typedef unsigned char uint8_t;
typedef short int16_t;
typedef unsigned short uint16_t;
typedef int int32_t;
typedef unsigned int uint32_t;
typedef long long int64_t;
typedef unsigned long long uint64_t;
typedef unsigned long size_t;
#endif

#include "opcodes.h"

#define LDS __attribute__((address_space(3)))

namespace polar {
namespace {

__host__ __device__ constexpr int lds_align16(int x) { return (x + 15) & ~15; }

typedef short s2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// Lane movement: lane i receives x from lane i + H.  Valid for every lane
// whose bit H is clear (the lanes that need the partner element).
// ---------------------------------------------------------------------------
template <int H>
__device__ __forceinline__ uint32_t from_up(uint32_t x) {
  static_assert(H == 1 || H == 2 || H == 4 || H == 8 || H == 16 || H == 32, "lane distance");
  if constexpr (H <= 8) {
    // row_shl:H; lanes with no source in their row read 0 (bound_ctrl),
    // so no register has to be zeroed first
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x100 + H, 0xf, 0xf, true);
  } else {
    // the swap's second operand only receives; leave it undefined so that
    // x needs one copy, not two
    uint32_t any;
    asm("" : "=v"(any));
    if constexpr (H == 16) return __builtin_amdgcn_permlane16_swap(x, any, false, false)[1];
    else return __builtin_amdgcn_permlane32_swap(x, any, false, false)[1];
  }
}
template <int H>
__device__ __forceinline__ float from_up(float x) {
  return __uint_as_float(from_up<H>(__float_as_uint(x)));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__builtin_amdgcn_ballot_w64(p); }
// Per lane: -x if bit `lane` of the wave-uniform mask m is set, else x (one
// v_cndmask with the mask as its SGPR-pair condition and the negation as a
// source modifier).
__device__ __forceinline__ float negate_lanes(uint64_t m, float x) {
  // the mask is wave-uniform; readfirstlane tells the compiler so (and
  // costs nothing when it already lives in scalar registers)
  const uint64_t mu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32) |
                      (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)m);
  float r;
  asm("v_cndmask_b32_e64 %0, %1, -%1, %2" : "=v"(r) : "v"(x), "s"(mu));
  return r;
}
__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
// Lane J of v set to the wave-uniform x (v_writelane_b32), other lanes kept.
template <int J>
__device__ __forceinline__ uint32_t write_lane(uint32_t v, uint32_t x) {
  asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(x), "i"(J));
  return v;
}
__device__ __forceinline__ float rflf(float x) { return __uint_as_float(rfl(__float_as_uint(x))); }
// Orders the wave's LDS traffic across lanes and keeps the compiler from
// moving memory operations over op boundaries.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// f(integral_constant<int, 0>) .. f(integral_constant<int, N-1>)
template <int V>
struct int_c {
  static constexpr int value = V;
};
template <int N, int I = 0, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(int_c<I>{});
    static_for<N, I + 1>(f);
  }
}

__device__ __forceinline__ uint64_t low_mask(int bits) { return bits >= 64 ? ~0ull : ((1ull << bits) - 1ull); }

// u = x G on up to 64 bits: x[i] ^= x[i+h] for every i with bit h clear.
__device__ __forceinline__ uint64_t transform64(uint64_t x, int size) {
  if (size > 1) x ^= (x >> 1) & 0x5555555555555555ull;
  if (size > 2) x ^= (x >> 2) & 0x3333333333333333ull;
  if (size > 4) x ^= (x >> 4) & 0x0F0F0F0F0F0F0F0Full;
  if (size > 8) x ^= (x >> 8) & 0x00FF00FF00FF00FFull;
  if (size > 16) x ^= (x >> 16) & 0x0000FFFF0000FFFFull;
  if (size > 32) x ^= (x >> 32) & 0x00000000FFFFFFFFull;
  return x;
}

// transform64 of a node of at most 32 bits, in 32-bit scalar operations
template <int NV>
__device__ __forceinline__ uint64_t transform_node(uint64_t x) {
  if constexpr (NV <= 32) {
    uint32_t y = (uint32_t)x;
    if constexpr (NV > 1) y ^= (y >> 1) & 0x55555555u;
    if constexpr (NV > 2) y ^= (y >> 2) & 0x33333333u;
    if constexpr (NV > 4) y ^= (y >> 4) & 0x0F0F0F0Fu;
    if constexpr (NV > 8) y ^= (y >> 8) & 0x00FF00FFu;
    if constexpr (NV > 16) y ^= (y >> 16) & 0x0000FFFFu;
    return (uint64_t)y;
  } else {
    return transform64(x, NV);
  }
}

__device__ __forceinline__ uint32_t transform32(uint32_t x) {
  x ^= (x >> 1) & 0x55555555u;
  x ^= (x >> 2) & 0x33333333u;
  x ^= (x >> 4) & 0x0F0F0F0Fu;
  x ^= (x >> 8) & 0x00FF00FFu;
  x ^= (x >> 16) & 0x0000FFFFu;
  return x;
}

// ---------------------------------------------------------------------------
// int8 LLRs on packed 16-bit lanes.  A 32-bit word holds LLRs e0..e3; read
// as two 16-bit lanes it is (256 e1 + u(e0), 256 e3 + u(e2)), u = the byte
// as unsigned: the odd LLRs in the high bytes, the even ones as a noise byte
// below them ("garbled").  The even LLRs are moved up with a zero low byte
// ("clean": 256 e0, 256 e2).  A lane 256 v + n (0 <= n < 256) stands for v.
//
// min and max of such lanes give the min and max of the values, whatever
// the noise; 255 - x (saturating) stands for -v (channel -128 -> +127); so f
// = max(min(a, b), 255 - max(a, b)) takes clean or garbled operands and
// returns garbled ones, -128 read as -127 (eq. (1)).  g = b + s a needs a
// clean a (the noise would be multiplied) but takes a garbled b: the sum's
// noise stays below the high byte; it saturates to the 16-bit range and is
// clamped below at -32512, which is Listing 4's saturation to [-127, 127].
// Results are packed by their high bytes; no result reads as -128.
// ---------------------------------------------------------------------------
__device__ __forceinline__ s2 as_s2(uint32_t x) { return __builtin_bit_cast(s2, x); }
__device__ __forceinline__ uint32_t as_u(s2 x) { return __builtin_bit_cast(uint32_t, x); }
// LLRs e0, e2 of a word, clean
__device__ __forceinline__ s2 even_lanes(uint32_t w) { return as_s2(__builtin_amdgcn_perm(0u, w, 0x020c000cu)); }
// LLRs e1, e3 of a word, garbled (the word itself)
__device__ __forceinline__ s2 odd_lanes(uint32_t w) { return as_s2(w); }
// the word of four results: high bytes of the even and odd lanes
__device__ __forceinline__ uint32_t pack_eo(s2 even, s2 odd) {
  return __builtin_amdgcn_perm(as_u(odd), as_u(even), 0x07030501u);
}
// garbled -> clean
__device__ __forceinline__ s2 clean(s2 r) { return as_s2(as_u(r) & 0xFF00FF00u); }
// lower clamp of a saturated sum: [-32768, 32767] -> [-32512, 32767]
__device__ __forceinline__ s2 sat_lo(s2 r) {
  const s2 lo = {(short)-32512, (short)-32512};
  return __builtin_elementwise_max(r, lo);
}
// f: sgn(a) sgn(b) min(|a|, |b|) = max(min(a, b), -max(a, b))
__device__ __forceinline__ s2 fx(s2 a, s2 b) {
  const s2 c255 = {255, 255};
  return __builtin_elementwise_max(__builtin_elementwise_min(a, b),
                                   __builtin_elementwise_sub_sat(c255, __builtin_elementwise_max(a, b)));
}
// g: b + s a, s = +-1 per lane (-1 where beta_l = 1); a clean, b clean or
// garbled.  One multiply-add saturated to the 16-bit range (the product is
// exact), then the lower clamp.
__device__ __forceinline__ s2 gx(s2 a, s2 b, s2 s) {
  uint32_t d;
  asm("v_pk_mad_i16 %0, %1, %2, %3 clamp" : "=v"(d) : "v"(as_u(a)), "v"(as_u(s)), "v"(as_u(b)));
  return sat_lo(as_s2(d));
}
__device__ __forceinline__ s2 g0x(s2 a, s2 b) { return sat_lo(__builtin_elementwise_add_sat(b, a)); }
// channel value -128 read as -127 (clean or garbled lanes)
__device__ __forceinline__ s2 chanx(s2 a) { return sat_lo(a); }

// One word (4 LLRs) of f, g or g_0R from words A (alpha_v[i..i+3]) and B
// (alpha_v[i+h..i+h+3]); sg: the g sign lanes of the even and odd LLRs.
// CH: A and B are channel words (-128 possible).
template <uint32_t CODE, bool CH>
__device__ __forceinline__ uint32_t fg_word_i8(uint32_t A, uint32_t B, u32x2 sg) {
  s2 ae = even_lanes(A), be = even_lanes(B), ao = odd_lanes(A), bo = odd_lanes(B);
  if constexpr (CODE != DOP_F) {
    ao = clean(ao);  // a of g must be clean
    if constexpr (CH) {
      ae = chanx(ae);
      be = chanx(be);
      ao = chanx(ao);
      bo = chanx(bo);
    }
  }
  s2 re, ro;
  if constexpr (CODE == DOP_F) {
    re = fx(ae, be);
    ro = fx(ao, bo);
  } else if constexpr (CODE == DOP_G) {
    re = gx(ae, be, as_s2(sg[0]));
    ro = gx(ao, bo, as_s2(sg[1]));
  } else {
    re = g0x(ae, be);
    ro = g0x(ao, bo);
  }
  return pack_eo(re, ro);
}

// ---------------------------------------------------------------------------
// Arithmetic policies
// ---------------------------------------------------------------------------
struct PI8 {
  typedef int8_t Chan;
  static constexpr int ELEM = 1;
  static __device__ __forceinline__ float clamp32(float x) { return __builtin_amdgcn_fmed3f(x, -127.0f, 127.0f); }
  static __device__ __forceinline__ float chan(int v) { return (float)(v < -127 ? -127 : v); }
  static __device__ __forceinline__ int8_t to_chan(float v) { return (int8_t)(int)v; }
};

struct PF32 {
  typedef float Chan;
  static constexpr int ELEM = 4;
  static __device__ __forceinline__ float clamp32(float x) { return x; }
  static __device__ __forceinline__ float to_chan(float v) { return v; }
};

__device__ __forceinline__ float fmin_sum(float x, float y) { return fmaxf(fminf(x, y), fminf(-x, -y)); }

// ---------------------------------------------------------------------------
// Per-wave decoder
// ---------------------------------------------------------------------------
template <class P>
struct Dec {
  typedef typename P::Chan Chan;

  int lane;
  int log2n;
  LDS unsigned char* alpha;   // stage s (7 <= s < log2n) at alpha + (2^s - 128) * ELEM
  LDS uint32_t* beta;         // N bits, natural order
  LDS uint32_t* lut;          // int8 g signs: 16 entries of two +-1 pairs
  __amdgpu_buffer_rsrc_t chr; // channel row
  Chan* tr;                   // trace row (global) or null
  uint8_t* row;               // output row (global)
  int row_bytes;

  float a[7];                 // stages 0..6
  uint64_t win;               // beta of the current 64-aligned block
  uint64_t acc;               // output accumulator
  int fill;                   // bits held in acc
  int words_out;              // 64-bit output words stored so far
  uint64_t pend_v;            // bits the last op wants appended ...
  int pend_n;                 // ... and how many (0: none)

  __device__ __forceinline__ LDS unsigned char* stage(int s) const { return alpha + ((1 << s) - 128) * P::ELEM; }

  // g sign pairs of the 4 elements whose beta_l bits are bits 4k..4k+3 of
  // `bits` (int8 table entry; one bit-field extract and one address add)
  __device__ __forceinline__ u32x2 gsigns(uint32_t bits, int k) const {
    // (the compiler turns a plain field extract into shift, mask and add)
    uint32_t e;
    asm("v_bfe_u32 %0, %1, %2, 4" : "=v"(e) : "v"(bits), "i"(4 * k));
    return *(const LDS u32x2*)((const LDS unsigned char*)lut + 8 * e);
  }

  // ------------------------------------------------------------- output
  __device__ __forceinline__ void emit(uint64_t w) {
    const int idx = 8 * words_out + lane;
    if (lane < 8 && idx < row_bytes) row[idx] = (uint8_t)(w >> (8 * lane));
    ++words_out;
  }
  // append the low n bits of v (1 <= n <= 64; higher bits must be 0)
  __device__ __forceinline__ void append(uint64_t v, int n) {
    acc |= v << fill;
    const int nf = fill + n;
    if (nf >= 64) {
      emit(acc);
      acc = fill ? (v >> (64 - fill)) : 0ull;
      fill = nf - 64;
    } else {
      fill = nf;
    }
  }

  // Bits recorded by the last small leaf or repetition node (one copy of
  // the append code in the interpreter loop).
  __device__ __forceinline__ void settle() {
    if (pend_n) {
      append(pend_v, pend_n);
      pend_n = 0;
    }
  }

  // Dword d of the output stream of a leaf whose u is staged as 32-bit
  // words at st: the fill bits held in acc, then u bits from skip on.  A
  // dword past the node reads staged words past it, which only feed bits
  // that are cut off (the caller masks them).
  __device__ __forceinline__ uint32_t stream_dword(const LDS uint32_t* st, int d, int skip) const {
    const int s = 32 * d - fill + skip;  // u bit at the dword's bit 0
    if (32 * d >= fill) return __builtin_amdgcn_alignbit(st[(s >> 5) + 1], st[s >> 5], s & 31);
    const int k = fill - 32 * d;  // acc bits in this dword (d = 0 or 1)
    const uint32_t a = (uint32_t)(acc >> (32 * d));
    if (k >= 32) return a;
    return (a & ((1u << k) - 1u)) | (__builtin_amdgcn_alignbit(st[1], st[0], skip) << k);
  }

  // ------------------------------------------------- nodes of size <= 64
  template <int S>
  __device__ __forceinline__ void small_fg(uint32_t code, int o) {
    constexpr int H = 1 << (S - 1);
    const float x = a[S];
    const float y = from_up<H>(x);
    if (code == DOP_F) {
      a[S - 1] = fmin_sum(x, y);
    } else if (code == DOP_G) {
      a[S - 1] = P::clamp32(y + negate_lanes(win >> (o & 63), x));
    } else {
      a[S - 1] = P::clamp32(y + x);
    }
  }

  // SPC correction index of a node of size NV <= 64 held one LLR per lane:
  // the lowest lane among lanes < NV of least |x| (Listing 2's first-match
  // search).  int8 codes: every value is an integer below 2^7, so the low 16
  // bits of |x|'s float encoding are zero and hold the lane, and one minimum
  // over the keys gives both; float codes: the minimum, then the first lane
  // attaining it.
  template <int NV>
  __device__ __forceinline__ int spc_min_lane(float x) const {
    if constexpr (P::ELEM == 1) {
      uint32_t key = (__float_as_uint(x) & 0x7fffffffu) | (uint32_t)lane;
      if constexpr (NV < 64) key = lane < NV ? key : 0xffffffffu;
      if constexpr (NV >= 64) key = min(key, from_up<32>(key));
      if constexpr (NV >= 32) key = min(key, from_up<16>(key));
      if constexpr (NV >= 16) key = min(key, from_up<8>(key));
      if constexpr (NV >= 8) key = min(key, from_up<4>(key));
      if constexpr (NV >= 4) key = min(key, from_up<2>(key));
      if constexpr (NV >= 2) key = min(key, from_up<1>(key));
      return (int)(rfl(key) & 63u);
    } else {
      float v = lane < NV ? fabsf(x) : 3.0e38f;
      if constexpr (NV >= 64) v = fminf(v, from_up<32>(v));
      if constexpr (NV >= 32) v = fminf(v, from_up<16>(v));
      if constexpr (NV >= 16) v = fminf(v, from_up<8>(v));
      if constexpr (NV >= 8) v = fminf(v, from_up<4>(v));
      if constexpr (NV >= 4) v = fminf(v, from_up<2>(v));
      if constexpr (NV >= 2) v = fminf(v, from_up<1>(v));
      const float mn = rflf(v);
      const uint64_t cand = ballot(lane < NV && fabsf(x) == mn);
      return __ffsll((unsigned long long)cand) - 1;
    }
  }

  __device__ __forceinline__ void set_win(int off, uint64_t m, uint64_t bits) {
    win = (win & ~(m << off)) | (bits << off);
  }

  template <int S>
  __device__ __forceinline__ void small_leaf(uint32_t code, int o) {
    constexpr int NV = 1 << S;
    const int off = o & 63;
    const uint64_t m = low_mask(NV);
    const float x = a[S];
    if (tr && lane < NV) tr[o + lane] = P::to_chan(x);
    uint64_t hd = ballot(x < 0.0f) & m;
    if (code == DOP_R1) {
      set_win(off, m, hd);
      pend_v = transform_node<NV>(hd);
      pend_n = NV;
    } else if (code == DOP_REP) {
      float s = x;
      if constexpr (NV >= 64) s += from_up<32>(s);
      if constexpr (NV >= 32) s += from_up<16>(s);
      if constexpr (NV >= 16) s += from_up<8>(s);
      if constexpr (NV >= 8) s += from_up<4>(s);
      if constexpr (NV >= 4) s += from_up<2>(s);
      if constexpr (NV >= 2) s += from_up<1>(s);
      const bool bit = rflf(s) < 0.0f;
      set_win(off, m, bit ? m : 0ull);
      pend_v = bit ? 1ull : 0ull;
      pend_n = 1;
    } else {  // DOP_SPC
      if (__popcll(hd) & 1) hd ^= 1ull << spc_min_lane<NV>(x);
      set_win(off, m, hd);
      pend_v = transform_node<NV>(hd) >> 1;
      pend_n = NV - 1;
    }
  }

  // Fused leaf-pair node of size NV = 2^S (DOP_P01 .. DOP_REPR1): the left
  // child (size H = NV/2) is Rate-0 or a repetition node, the right child
  // Rate-1 or SPC.  Same arithmetic as f, the repetition sum, g, the
  // right leaf and the combine run as separate ops; the node's beta goes to
  // the window and its information bits (left leaf first) to the output in
  // one step each.
  template <int S>
  __device__ __forceinline__ void small_pair(uint32_t code, int o) {
    constexpr int NV = 1 << S, H = NV >> 1;
    const int off = o & 63;
    const uint64_t m = low_mask(H);
    const bool rep_left = code == DOP_REPSPC || code == DOP_REPR1;
    const bool spc_right = code == DOP_REPSPC || code == DOP_0SPC;
    const float x = a[S];
    const float y = from_up<H>(x);
    bool rep = false;
    float g;
    if (rep_left) {
      const float f = fmin_sum(x, y);
      if (tr && lane < H) tr[o + lane] = P::to_chan(f);
      float s = f;
      if constexpr (H >= 32) s += from_up<16>(s);
      if constexpr (H >= 16) s += from_up<8>(s);
      if constexpr (H >= 8) s += from_up<4>(s);
      if constexpr (H >= 4) s += from_up<2>(s);
      if constexpr (H >= 2) s += from_up<1>(s);
      rep = rflf(s) < 0.0f;
      g = P::clamp32(y + (rep ? -x : x));
    } else {
      g = P::clamp32(y + x);
    }
    if (tr && lane < H) tr[o + H + lane] = P::to_chan(g);
    uint64_t hd = ballot(g < 0.0f) & m;
    uint64_t out;
    int nout;
    if (spc_right) {
      if (__popcll(hd) & 1) hd ^= 1ull << spc_min_lane<H>(g);
      out = transform_node<H>(hd) >> 1;
      nout = H - 1;
    } else {
      out = transform_node<H>(hd);
      nout = H;
    }
    set_win(off, low_mask(NV), (((rep ? m : 0ull) ^ hd) | (hd << H)));
    if (rep_left) {
      pend_v = (rep ? 1ull : 0ull) | (out << 1);
      pend_n = nout + 1;
    } else {
      pend_v = out;
      pend_n = nout;
    }
  }

  __device__ __forceinline__ void small_combine(uint32_t code, int S, int o) {
    const int h = 1 << (S - 1);
    const int off = o & 63;
    const uint64_t m = low_mask(h);
    const uint64_t r = (win >> (off + h)) & m;
    if (code == DOP_C)
      win ^= r << off;
    else if (code == DOP_C0R)
      set_win(off, m, r);
    else
      win &= ~(m << (off + h));
  }

  // ------------------------------------------ big nodes: beta in LDS bits
  __device__ __forceinline__ void big_combine(uint32_t code, int S, int o) {
    const int h = 1 << (S - 1);
    const int words = h >> 5;
    LDS uint32_t* l = beta + (o >> 5);
    LDS uint32_t* r = beta + ((o + h) >> 5);
    for (int j = lane; j < words; j += 64) {
      if (code == DOP_C)
        l[j] ^= r[j];
      else if (code == DOP_C0R)
        l[j] = r[j];
      else
        r[j] = 0u;
    }
  }

  // window of a finished size-64 node -> LDS bits
  __device__ __forceinline__ void flush(int o) {
    if (lane < 2) beta[(o >> 5) + lane] = (uint32_t)(win >> (32 * lane));
  }

  // ---------------------------------------- stage 7 -> stage 6 (registers)
  __device__ __forceinline__ float load7(int i) {
    // element i of the input of an op at stage 7 (LDS stage 7 or channel)
    if (log2n == 7) {
      if constexpr (P::ELEM == 1)
        return P::chan((int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(chr, i, 0, 0));
      else
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * i, 0, 0));
    }
    if constexpr (P::ELEM == 1)
      return (float)*(const LDS int8_t*)(stage(7) + i);
    else
      return *(const LDS float*)(stage(7) + 4 * i);
  }

  __device__ __forceinline__ void fg7(uint32_t code) {
    const float x = load7(lane), y = load7(lane + 64);
    if (code == DOP_F)
      a[6] = fmin_sum(x, y);
    else if (code == DOP_G)
      a[6] = P::clamp32(y + negate_lanes(win, x));  // beta of the left size-64 child
    else
      a[6] = P::clamp32(y + x);
  }

  // ------------------------------------------------- big F / G / G_0R
  // int8: lane chunks of CB bytes (CB = 16, or 4 for nodes below 4096).
  template <int CB, bool CH, uint32_t CODE>
  __device__ __forceinline__ void i8_fg(int S, int o) {
    const int h = 1 << (S - 1);
    const LDS unsigned char* in = stage(S);
    LDS unsigned char* out = stage(S - 1);
    constexpr int NW = CB / 4;
    for (int base = 0; base < h; base += 64 * CB) {
      const int i0 = base + lane * CB;
      if (i0 < h) {
        uint32_t A[NW], B[NW], R[NW];
        if constexpr (CH) {
          if constexpr (CB == 16) {
            const u32x4 va = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, i0, 0, 0));
            const u32x4 vb = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, i0 + h, 0, 0));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              A[k] = va[k];
              B[k] = vb[k];
            }
          } else {
            A[0] = __builtin_amdgcn_raw_buffer_load_b32(chr, i0, 0, 0);
            B[0] = __builtin_amdgcn_raw_buffer_load_b32(chr, i0 + h, 0, 0);
          }
        } else {
          if constexpr (CB == 16) {
            const u32x4 va = *(const LDS u32x4*)(in + i0);
            const u32x4 vb = *(const LDS u32x4*)(in + i0 + h);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              A[k] = va[k];
              B[k] = vb[k];
            }
          } else {
            A[0] = *(const LDS uint32_t*)(in + i0);
            B[0] = *(const LDS uint32_t*)(in + i0 + h);
          }
        }
        uint32_t bb = 0;
        if constexpr (CODE == DOP_G) bb = beta[(o + i0) >> 5] >> ((o + i0) & 31);
#pragma unroll
        for (int k = 0; k < NW; ++k) {
          u32x2 sg = {0u, 0u};
          if constexpr (CODE == DOP_G) sg = gsigns(bb, k);
          R[k] = fg_word_i8<CODE, CH>(A[k], B[k], sg);
        }
        if constexpr (CB == 16)
          *(LDS u32x4*)(out + i0) = (u32x4){R[0], R[1], R[2], R[3]};
        else
          *(LDS uint32_t*)(out + i0) = R[0];
      }
    }
  }

  // float: lane chunks of 4 values (16 bytes).
  template <bool CH, uint32_t CODE>
  __device__ __forceinline__ void f32_fg(int S, int o) {
    const int h = 1 << (S - 1);
    const LDS float* in = (const LDS float*)stage(S);
    LDS float* out = (LDS float*)stage(S - 1);
    for (int base = 0; base < h; base += 256) {
      const int i0 = base + lane * 4;
      if (i0 < h) {
        float A[4], B[4], R[4];
        u32x4 va, vb;
        if constexpr (CH) {
          va = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, 4 * i0, 0, 0));
          vb = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, 4 * (i0 + h), 0, 0));
        } else {
          va = *(const LDS u32x4*)(in + i0);
          vb = *(const LDS u32x4*)(in + i0 + h);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          A[k] = __uint_as_float(va[k]);
          B[k] = __uint_as_float(vb[k]);
        }
        uint32_t bb = 0;
        if constexpr (CODE == DOP_G) bb = beta[(o + i0) >> 5] >> ((o + i0) & 31);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if constexpr (CODE == DOP_F)
            R[k] = fmin_sum(A[k], B[k]);
          else if constexpr (CODE == DOP_G)  // b + (-a) is exactly b - a
            R[k] = __fadd_rn(B[k], __uint_as_float(__float_as_uint(A[k]) ^ ((bb << (31 - k)) & 0x80000000u)));
          else
            R[k] = __fadd_rn(B[k], A[k]);
        }
        *(LDS u32x4*)(out + i0) =
            (u32x4){__float_as_uint(R[0]), __float_as_uint(R[1]), __float_as_uint(R[2]), __float_as_uint(R[3])};
      }
    }
  }

  template <uint32_t CODE>
  __device__ __forceinline__ void big_fg_code(int S, int o) {
    const bool ch = S == log2n;
    if constexpr (P::ELEM == 1) {
      if (S >= 12) {
        if (ch)
          i8_fg<16, true, CODE>(S, o);
        else
          i8_fg<16, false, CODE>(S, o);
      } else {
        if (ch)
          i8_fg<4, true, CODE>(S, o);
        else
          i8_fg<4, false, CODE>(S, o);
      }
    } else {
      if (ch)
        f32_fg<true, CODE>(S, o);
      else
        f32_fg<false, CODE>(S, o);
    }
  }

  __device__ __forceinline__ void big_fg(uint32_t code, int S, int o) {
    if (S == 7) {
      fg7(code);
      return;
    }
    if (code == DOP_F)
      big_fg_code<DOP_F>(S, o);
    else if (code == DOP_G)
      big_fg_code<DOP_G>(S, o);
    else
      big_fg_code<DOP_G0R>(S, o);
  }

  // ------------------------------------------------------- big leaves
  // Elements i0 .. i0+3 of the input of a leaf at stage S (LDS or channel).
  __device__ __forceinline__ void leaf_quad(int S, int i0, float* v) {
    if constexpr (P::ELEM == 1) {
      uint32_t w;
      if (S == log2n)
        w = __builtin_amdgcn_raw_buffer_load_b32(chr, i0, 0, 0);
      else
        w = *(const LDS uint32_t*)(stage(S) + i0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int x = (int)(int8_t)(w >> (8 * k));
        v[k] = (float)(x < -127 ? -127 : x);
      }
    } else {
      u32x4 q;
      if (S == log2n)
        q = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, 4 * i0, 0, 0));
      else
        q = *(const LDS u32x4*)(stage(S) + 4 * i0);
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = __uint_as_float(q[k]);
    }
  }

  __device__ __forceinline__ void big_leaf(uint32_t code, int S, int o) {
    const int nv = 1 << S;
    LDS uint32_t* bw = beta + (o >> 5);
    if (code == DOP_REP) {
      float s;
      if constexpr (P::ELEM == 1) {
        // integers: every partial sum is exact, so the order is free
        int acc_i = 0;
        for (int i0 = 4 * lane; i0 < nv; i0 += 256) {
          float v[4];
          leaf_quad(S, i0, v);
          if (tr)
            for (int k = 0; k < 4; ++k) tr[o + i0 + k] = P::to_chan(v[k]);
          acc_i += (int)v[0] + (int)v[1] + (int)v[2] + (int)v[3];
        }
        s = (float)acc_i;
        s += __shfl_xor(s, 32, 64);
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 8, 64);
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 1, 64);
      } else {
        s = rep_halving_f32(S, o);
      }
      const bool bit = rflf(s) < 0.0f;
      for (int j = lane; j < (nv >> 5); j += 64) bw[j] = bit ? ~0u : 0u;
      pend_v = bit ? 1ull : 0ull;
      pend_n = 1;
      return;
    }
    switch (S) {
      case 7: leaf_r1spc<7>(code, o); break;
      case 8: leaf_r1spc<8>(code, o); break;
      case 9: leaf_r1spc<9>(code, o); break;
      case 10: leaf_r1spc<10>(code, o); break;
      case 11: leaf_r1spc<11>(code, o); break;
      case 12: leaf_r1spc<12>(code, o); break;
      case 13: leaf_r1spc<13>(code, o); break;
      case 14: leaf_r1spc<14>(code, o); break;
      default: leaf_r1spc<15>(code, o); break;
    }
  }

  // Hard decisions (eq. (4)) of elements i0 .. i0+31 of the input of a leaf
  // at stage S: bit k is 1 iff element i0 + k is negative.
  template <int S, bool CH>
  __device__ __forceinline__ uint32_t hd32(int i0) {
    uint32_t d = 0;
    if constexpr (P::ELEM == 1) {
      u32x4 q0, q1;
      if constexpr (CH) {
        q0 = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, i0, 0, 0));
        q1 = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, i0 + 16, 0, 0));
      } else {
        q0 = *(const LDS u32x4*)(stage(S) + i0);
        q1 = *(const LDS u32x4*)(stage(S) + i0 + 16);
      }
      // the sign bit of each byte, gathered four at a time by a dot product
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        d |= __builtin_amdgcn_udot4((q0[k] >> 7) & 0x01010101u, 0x08040201u, 0u, false) << (4 * k);
        d |= __builtin_amdgcn_udot4((q1[k] >> 7) & 0x01010101u, 0x08040201u, 0u, false) << (16 + 4 * k);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        u32x4 v;
        if constexpr (CH)
          v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(chr, 4 * (i0 + 4 * q), 0, 0));
        else
          v = *(const LDS u32x4*)(stage(S) + 4 * (i0 + 4 * q));
#pragma unroll
        for (int k = 0; k < 4; ++k) d |= (__uint_as_float(v[k]) < 0.0f ? 1u : 0u) << (4 * q + k);
      }
    }
    return d;
  }

  // Element i of the input of a leaf at stage S (int8: -128 read as -127).
  template <int S>
  __device__ __forceinline__ float leaf_elem(int i) {
    if constexpr (P::ELEM == 1) {
      int x;
      if (S == log2n)
        x = (int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(chr, i, 0, 0);
      else
        x = (int)*(const LDS int8_t*)(stage(S) + i);
      return (float)(x < -127 ? -127 : x);
    } else {
      if (S == log2n) return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * i, 0, 0));
      return ((const LDS float*)stage(S))[i];
    }
  }

  // SPC correction index (Listing 2): the lowest index among the elements of
  // least magnitude.  Wave-uniform result.
  template <int S>
  __device__ __forceinline__ int spc_argmin() {
    constexpr int NV = 1 << S;
    float best = 3.0e38f;
    int bi = 0x7fffffff;
#pragma unroll 8
    for (int i = lane; i < NV; i += 64) {
      const float m = fabsf(leaf_elem<S>(i));
      if (m < best) {  // indices grow, so the first of equal values stays
        best = m;
        bi = i;
      }
    }
    return argmin_reduce(best, bi);
  }

  // Wave-wide (minimum, lowest index attaining it) from per-lane candidates.
  __device__ __forceinline__ int argmin_reduce(float best, int bi) {
    float v = best;
    v = fminf(v, __shfl_xor(v, 32, 64));
    v = fminf(v, __shfl_xor(v, 16, 64));
    v = fminf(v, __shfl_xor(v, 8, 64));
    v = fminf(v, __shfl_xor(v, 4, 64));
    v = fminf(v, __shfl_xor(v, 2, 64));
    v = fminf(v, __shfl_xor(v, 1, 64));
    int idx = best == v ? bi : 0x7fffffff;
    idx = min(idx, __shfl_xor(idx, 32, 64));
    idx = min(idx, __shfl_xor(idx, 16, 64));
    idx = min(idx, __shfl_xor(idx, 8, 64));
    idx = min(idx, __shfl_xor(idx, 4, 64));
    idx = min(idx, __shfl_xor(idx, 2, 64));
    idx = min(idx, __shfl_xor(idx, 1, 64));
    return (int)rfl((uint32_t)idx);
  }

  // The node's beta words from hard decisions: lane j gets words j, j+64, ...
  template <int S, bool CH, int PER>
  __device__ __forceinline__ void hd_words(uint32_t* wd) {
    constexpr int NW = 1 << (S - 5);
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int j = lane + 64 * m;
      wd[m] = 0u;
      if (NW >= 64 || j < NW) wd[m] = hd32<S, CH>(32 * j);
    }
  }

  // Words w (bit D of the lane index clear) ^= word w + D, D < 64 words.
  template <int D, int PER>
  __device__ __forceinline__ void xor_up_lanes(uint32_t* wd) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      if constexpr (D == 4 || D == 8) {
        // the lanes with bit D clear are banks 0 and 2 (D = 4) or 0 and 1
        // (D = 8) of each 16-lane row: a bank-masked DPP move reaches only
        // them, the others read 0
        wd[m] ^= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wd[m], 0x100 + D, 0xf, D == 4 ? 0x5 : 0x3, false);
      } else {
        const uint32_t p = from_up<D>(wd[m]);
        if ((lane & D) == 0) wd[m] ^= p;
      }
    }
  }

  // Rate-1 or SPC leaf of size 2^S >= 128.  Lane j holds beta words
  // j, j + 64, ... (32 elements each) in registers: hard decisions, the SPC
  // parity check and correction (Sec. II-E), the words to the beta array,
  // then u = beta G in registers and the information bits (all of u, or u
  // without u_0 for SPC) to the output, 64-bit words in parallel.
  // st_stage: an LDS alpha stage free at this leaf, of at least 2^S / 8
  // bytes, used as scratch (default: the stage below the leaf).
  // Rate-1 or SPC leaf of 128..512 int8 LLRs: lane L reads elements
  // L + 64m, so the hard decisions of each 64 consecutive elements are one
  // ballot, in index order; the parity and the SPC correction are scalar
  // work on those 64-bit words, which then go to lanes (word j to lane j) for
  // the beta array, u = beta G and the output.  The SPC correction takes the least
  // key |alpha_i| * 512 + i (lowest index among equal magnitudes, Listing 2).
  template <int S>
  __device__ __forceinline__ void leaf_ballot(uint32_t code, int o, int st_stage) {
    constexpr int NV = 1 << S;
    constexpr int NM = NV / 64;  // 64-bit words of hard decisions
    constexpr int NW = NV / 32;
    static_assert(P::ELEM == 1 && S >= 7 && S <= 9, "int8 leaves of 128..512 LLRs");
    int x[NM];
    uint64_t hd[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      if (S == log2n)
        x[m] = max((int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(chr, lane + 64 * m, 0, 0), -127);
      else
        x[m] = (int)*(const LDS int8_t*)(stage(S) + lane + 64 * m);
      hd[m] = ballot(x[m] < 0);
    }
    if (tr)
#pragma unroll
      for (int m = 0; m < NM; ++m) tr[o + lane + 64 * m] = (Chan)x[m];
    if (code == DOP_SPC) {
      int par = 0;
#pragma unroll
      for (int m = 0; m < NM; ++m) par ^= __popcll(hd[m]);
      if (par & 1) {
        uint32_t key = 0xffffffffu;
#pragma unroll
        for (int m = 0; m < NM; ++m) key = min(key, ((uint32_t)abs(x[m]) << 9) | (uint32_t)(lane + 64 * m));
        key = min(key, from_up<32>(key));
        key = min(key, from_up<16>(key));
        key = min(key, from_up<8>(key));
        key = min(key, from_up<4>(key));
        key = min(key, from_up<2>(key));
        key = min(key, from_up<1>(key));
        const int idx = (int)(rfl(key) & 511u);
#pragma unroll
        for (int m = 0; m < NM; ++m)
          if ((idx >> 6) == m) hd[m] ^= 1ull << (idx & 63);
      }
    }
    // beta words to LDS: lane j stores word j
    LDS uint32_t* bw = beta + (o >> 5);
    uint32_t w;
    asm("" : "=v"(w));  // lanes >= NW are never read: no initial value
    static_for<NW>([&](auto j) { w = write_lane<j.value>(w, rfl((uint32_t)(hd[j.value >> 1] >> (32 * (j.value & 1))))); });
    if (lane < NW) bw[lane] = w;
    // u = beta G and the output bits from the words in lanes (vector work,
    // as for the wider leaves)
    finish_leaf<S, 1>(&w, code, (LDS uint32_t*)stage(st_stage));
  }

  template <int S>
  __device__ __forceinline__ void leaf_r1spc(uint32_t code, int o, int st_stage = S - 1) {
    if constexpr (P::ELEM == 1 && S >= 7 && S <= 9) {
      leaf_ballot<S>(code, o, st_stage);
      return;
    }
    constexpr int NV = 1 << S;
    constexpr int NW = NV >> 5;                 // 32-bit words: 4 .. 1024
    constexpr int PER = NW >= 64 ? NW / 64 : 1; // words per lane
    LDS uint32_t* bw = beta + (o >> 5);
    uint32_t wd[PER];
    if (S == log2n)
      hd_words<S, true, PER>(wd);
    else
      hd_words<S, false, PER>(wd);
    int par = 0;
#pragma unroll
    for (int m = 0; m < PER; ++m) par ^= __popc(wd[m]);
    if (tr)
      for (int i = lane; i < NV; i += 64) tr[o + i] = P::to_chan(leaf_elem<S>(i));
    if (code == DOP_SPC && (__popcll(ballot((par & 1) != 0)) & 1)) {
      const int idx = spc_argmin<S>();
      const int jw = idx >> 5;
      if ((jw & 63) == lane) {
#pragma unroll
        for (int m = 0; m < PER; ++m)
          if (m == (jw >> 6)) wd[m] ^= 1u << (idx & 31);
      }
    }
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int j = lane + 64 * m;
      if (NW >= 64 || j < NW) bw[j] = wd[m];
    }
    finish_leaf<S, PER>(wd, code, (LDS uint32_t*)stage(st_stage));
  }

  // u = beta G of a Rate-1 or SPC leaf of size 2^S from its beta words in
  // registers (lane j holds words j, j + 64, ...), and its information bits
  // (all of u, or u without u_0 for SPC) to the output.  st: LDS scratch of
  // at least 2^S / 8 bytes.
  template <int S, int PER>
  __device__ __forceinline__ void finish_leaf(uint32_t* wd, uint32_t code, LDS uint32_t* st) {
    constexpr int NV = 1 << S;
    constexpr int NW = NV >> 5;
    // u = beta G_NV: the levels inside a word, across lanes, across registers
#pragma unroll
    for (int m = 0; m < PER; ++m) wd[m] = transform32(wd[m]);
    if constexpr (NW > 1) xor_up_lanes<1, PER>(wd);
    if constexpr (NW > 2) xor_up_lanes<2, PER>(wd);
    if constexpr (NW > 4) xor_up_lanes<4, PER>(wd);
    if constexpr (NW > 8) xor_up_lanes<8, PER>(wd);
    if constexpr (NW > 16) xor_up_lanes<16, PER>(wd);
    if constexpr (NW > 32) xor_up_lanes<32, PER>(wd);
#pragma unroll
    for (int dm = 1; dm < PER; dm <<= 1)
#pragma unroll
      for (int m = 0; m < PER; ++m)
        if ((m & dm) == 0) wd[m] ^= wd[m + dm];
    const int skip = code == DOP_SPC ? 1 : 0;
    if constexpr (NW <= 4) {
      // 128 bits: through the scalar accumulator
      const uint64_t v0 = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)wd[0], 0) |
                          ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)wd[0], 1) << 32);
      const uint64_t v1 = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)wd[0], 2) |
                          ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)wd[0], 3) << 32);
      if (skip)
        append(v0 >> 1, 63);
      else
        append(v0, 64);
      append(v1, 64);
    } else {
      // stage u in st, then every lane builds whole output words
#pragma unroll
      for (int m = 0; m < PER; ++m)
        if (NW >= 64 || lane < NW) st[lane + 64 * m] = wd[m];
      wave_sync();
      const int total = fill + NV - skip;
      const int T = total >> 6;  // whole 64-bit words: inside the row, stored as dwords
      typedef uint32_t u32_unaligned __attribute__((aligned(1)));
      for (int d = lane; d < 2 * T; d += 64)
        *(u32_unaligned*)(row + 8 * words_out + 4 * d) = stream_dword(st, d, skip);
      const int nf = total & 63;
      uint64_t rest = 0;
      if (nf)  // same words in every lane
        rest = (((uint64_t)stream_dword(st, 2 * T + 1, skip) << 32) | stream_dword(st, 2 * T, skip)) & low_mask(nf);
      acc = ((uint64_t)rfl((uint32_t)(rest >> 32)) << 32) | rfl((uint32_t)rest);
      fill = nf;
      words_out += T;
    }
  }

  // Halving-tree repetition sum of a float leaf: the levels above 64 run in
  // place in the LDS buffer of the stage below (dead at a leaf), the last
  // 64 across lanes.
  __device__ __forceinline__ float rep_halving_f32(int S, int o) {
    const int nv = 1 << S;
    const bool ch = S == log2n;
    if (tr)
      for (int i = lane; i < nv; i += 64) {
        float v;
        if (ch)
          v = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * i, 0, 0));
        else
          v = ((const LDS float*)stage(S))[i];
        tr[o + i] = v;
      }
    float v;
    if (nv == 128) {
      // one level: lane i adds elements i and i + 64
      if (ch) {
        v = __fadd_rn(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * lane, 0, 0)),
                      __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * (lane + 64), 0, 0)));
      } else {
        v = __fadd_rn(((const LDS float*)stage(S))[lane], ((const LDS float*)stage(S))[lane + 64]);
      }
    } else {
      // nv >= 256: stage S-1 >= 7 exists and is dead at a leaf
      LDS float* buf = (LDS float*)stage(S - 1);
      // level m = nv: s_i = x_i + x_{i + nv/2}
      for (int i = lane; i < nv / 2; i += 64) {
        float x, y;
        if (ch) {
          x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * i, 0, 0));
          y = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * (i + nv / 2), 0, 0));
        } else {
          x = ((const LDS float*)stage(S))[i];
          y = ((const LDS float*)stage(S))[i + nv / 2];
        }
        buf[i] = __fadd_rn(x, y);
      }
      wave_sync();
      for (int m = nv / 2; m > 64; m >>= 1) {
        for (int i = lane; i < m / 2; i += 64) buf[i] = __fadd_rn(buf[i], buf[i + m / 2]);
        wave_sync();
      }
      v = buf[lane];
    }
    v = __fadd_rn(v, from_up<32>(v));
    v = __fadd_rn(v, from_up<16>(v));
    v = __fadd_rn(v, from_up<8>(v));
    v = __fadd_rn(v, from_up<4>(v));
    v = __fadd_rn(v, from_up<2>(v));
    v = __fadd_rn(v, from_up<1>(v));
    return v;
  }

  // ----------------------------------------------------------- dispatch
  __device__ __forceinline__ void small_op(uint32_t code, int S, int o) {
    if (code <= DOP_G0R) {
      switch (S) {
        case 1: small_fg<1>(code, o); break;
        case 2: small_fg<2>(code, o); break;
        case 3: small_fg<3>(code, o); break;
        case 4: small_fg<4>(code, o); break;
        case 5: small_fg<5>(code, o); break;
        default: small_fg<6>(code, o); break;
      }
    } else if (code <= DOP_CR0) {
      small_combine(code, S, o);
    } else if (code == DOP_FLUSH) {
      flush(o);
    } else if (is_pair_op(code)) {
      switch (S) {
        case 2: small_pair<2>(code, o); break;
        case 3: small_pair<3>(code, o); break;
        case 4: small_pair<4>(code, o); break;
        case 5: small_pair<5>(code, o); break;
        default: small_pair<6>(code, o); break;
      }
    } else {
      switch (S) {
        case 0: small_leaf<0>(code, o); break;
        case 1: small_leaf<1>(code, o); break;
        case 2: small_leaf<2>(code, o); break;
        case 3: small_leaf<3>(code, o); break;
        case 4: small_leaf<4>(code, o); break;
        case 5: small_leaf<5>(code, o); break;
        default: small_leaf<6>(code, o); break;
      }
    }
  }

  __device__ __forceinline__ void op(uint32_t w0) {
    const uint32_t code = w0 & 0xffu;
    const int S = (int)((w0 >> 8) & 0xffu);
    const int o = (int)(w0 >> 16);
    if (S <= 6)
      small_op(code, S, o);
    else if (code <= DOP_G0R)
      big_fg(code, S, o);
    else if (code <= DOP_CR0)
      big_combine(code, S, o);
    else
      big_leaf(code, S, o);
  }

  // one schedule step: the op, its output work, and op-to-op ordering
  __device__ __forceinline__ void step(uint32_t w0) {
    op(w0);
    settle();
    wave_sync();
  }

  // Sets up the decoder of frame `frame` in the LDS slot at `base`
  // (wave_lds_bytes(log2n, elem, nreg) bytes).
  __device__ __forceinline__ void init(LDS unsigned char* base, int lane_, int log2n_, int kbits,
                                       const Chan* llr, int frame, uint8_t* bits, Chan* trace, int nreg = 0) {
    const int n = 1 << log2n_;
    lane = lane_;
    log2n = log2n_;
    lut = (LDS uint32_t*)base;
    alpha = base + 128;
    beta = (LDS uint32_t*)(base + 128 + lds_align16(alpha_lds_bytes(log2n_, P::ELEM, nreg)));
    chr = __builtin_amdgcn_make_buffer_rsrc((void*)(llr + (size_t)frame * n), 0, n * (int)sizeof(Chan), 0x00020000);
    tr = trace ? trace + (size_t)frame * n : nullptr;
    row_bytes = (kbits + 7) / 8;
    row = bits + (size_t)frame * row_bytes;
    win = 0;
    acc = 0;
    fill = 0;
    words_out = 0;
    pend_v = 0;
    pend_n = 0;
#pragma unroll
    for (int s = 0; s < 7; ++s) a[s] = 0.0f;
    // g sign table: entry e (the beta bits of LLRs 0..3 of a word) -> the
    // +-1 lanes of the even LLRs (0, 2), then of the odd ones (1, 3)
    if (lane < 32) {
      const int e = lane >> 1, odd = lane & 1;
      const uint32_t b0 = (e >> odd) & 1u, b1 = (e >> (2 + odd)) & 1u;
      lut[lane] = (b0 ? 0x0000FFFFu : 0x00000001u) | (b1 ? 0xFFFF0000u : 0x00010000u);
    }
    // codes of at most 64 bits start in the registers of their root stage
    if (log2n <= 6) {
      float x;
      if constexpr (P::ELEM == 1)
        x = P::chan((int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(chr, lane, 0, 0));
      else
        x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(chr, 4 * lane, 0, 0));
      x = lane < n ? x : 0.0f;
      switch (log2n) {
        case 1: a[1] = x; break;
        case 2: a[2] = x; break;
        case 3: a[3] = x; break;
        case 4: a[4] = x; break;
        case 5: a[5] = x; break;
        default: a[6] = x; break;
      }
    }
    wave_sync();
  }

  // stores the last, partial output word
  __device__ __forceinline__ void finish() {
    if (fill > 0) emit(acc);
  }
};


// ---------------------------------------------------------------------------
// Decoder of the generated per-code kernels: every op word and the code
// length 2^L2N are compile-time constants, so each op is instantiated for
// its own stage and offset (Sec. III-B.4).  int8 codes may keep their NREG
// top alpha stages (L2N-1 down to L2N-NREG, each >= 2^11 LLRs) in registers
// instead of LDS, which cuts a frame's LDS footprint (N = 32768: 36.9 KB ->
// 12.3 KB) so that more frames share a compute unit; float codes of
// N >= 16384 keep one (L2N-2, below a virtual top stage).  Register stages use
// the chunked layout of the wide F/G ops: LLR e of stage s sits in lane
// (e >> 4) & 63, register 4 (e >> 10) + ((e >> 2) & 3), byte e & 3, so the
// pair e, e + 2^(s-1) of f and g is always lane-local.  A float register
// stage holds LLR e in lane (e >> 2) & 63, register 4 (e >> 8) + (e & 3).
// ---------------------------------------------------------------------------
template <int TOP, int NREG, int ELEM = 1>
struct RegStages {
  // register stages: TOP down to TOP - NREG + 1
  static constexpr bool has(int s) { return NREG > 0 && s <= TOP && s > TOP - NREG; }
  // first register of stage s: stage TOP first, then the next lower
  // (ELEM bytes per LLR: 256 / ELEM LLRs per register across the wave)
  static constexpr int base(int s) {
    int b = 0;
    for (int t = TOP; t > s; --t) b += ((1 << t) * ELEM) >> 8;
    return b;
  }
  static constexpr int total() { return NREG > 0 ? base(TOP - NREG) : 1; }
};

// VTOP = 1: the stage below the root (L2N-1) is never stored: the two ops
// that read it (f/g/g_0R of each child of the root) recompute it from the
// channel row with the root's op (fused_top), which frees its registers
// for the next two stages and keeps a frame within 128 VGPRs and 8.2 KB of
// LDS (N = 32768), four frames per SIMD.  Float codes of N >= 16384 use the
// virtual top stage and keep the stage below it (L2N-2) in registers
// (fused_top_f32 writes it), which cuts their LDS slot to about a quarter
// (N = 32768: 132 KB -> 36 KB, four frames per compute unit).  VMID = 1
// (float, N = 32768) does not store the stage below that register stage
// either (20 KB, eight frames per compute unit).
template <class P, int L2N, int NREG, int VTOP = 0, int VMID = 0>
struct DecU : Dec<P> {
  typedef Dec<P> B;
  typedef RegStages<L2N - 1 - VTOP, NREG, P::ELEM> R;
  static_assert(NREG == 0 || (P::ELEM == 1 ? L2N - VTOP - NREG >= 11 : (VTOP == 1 && NREG == 1 && L2N >= 14)),
                "register stages: int8 of >= 2^11 LLRs, or one float stage below a virtual top stage");
  static_assert(VTOP == 0 || (P::ELEM == 1 ? NREG >= 1 : NREG <= 1),
                "a virtual top stage feeds a register stage (int8) or the top float stage");
  static_assert(VMID == 0 || (P::ELEM == 4 && VTOP == 1 && NREG == 1 && L2N == 15),
                "a virtual stage below the float register stage: N = 32768 float codes");
  uint32_t rs[R::total()];

  // VMID = 1: the stage below the register stage (kVMid) is not stored
  // either: the ops of its nodes (step_mid) recompute their inputs from the
  // register stage with the parent's op
  static constexpr int kVMid = L2N - 1 - VTOP - NREG;
  // highest alpha stage in LDS: scratch for leaves at register stages
  static constexpr int kTopLds = L2N - 1 - VTOP - NREG - VMID;

  // Gives the registers of stage S new names before an op reads them, so
  // that no unpacked copies made by an earlier op on the same values stay
  // alive until a later one (f and g read the same LLRs, and the compiler
  // would otherwise share the unpacking between them).
  template <int S>
  __device__ __forceinline__ void launder() {
#pragma unroll
    for (int i = 0; i < ((1 << S) >> 8); ++i) asm volatile("" : "+v"(rs[R::base(S) + i]));
  }

  // ------------------------------------------------ wide F / G (int8)
  // One 32-bit word (4 LLRs) of f, g or g_0R; bits 4k..4k+3 of `bits`: its
  // beta_l bits (g).
  template <uint32_t CODE, bool CH>
  __device__ __forceinline__ uint32_t fg_word(uint32_t A, uint32_t Bw, uint32_t bits, int k) const {
    u32x2 sg = {0u, 0u};
    if constexpr (CODE == DOP_G) sg = this->gsigns(bits, k);
    return fg_word_i8<CODE, CH>(A, Bw, sg);
  }

  // f / g / g_0R of a node at stage S (8 <= S <= L2N) into stage S-1.  A lane
  // works on CB contiguous bytes of each half; batches of U iterations have
  // all their loads in flight before any arithmetic.  Sources: the channel
  // row, LDS or register stages; destinations: LDS or register stages.
  template <int S, uint32_t CODE>
  __device__ __forceinline__ void fg_i8(int o) {
    constexpr int H = 1 << (S - 1);
    constexpr bool CH = S == L2N;
    constexpr bool SREG = R::has(S), DREG = R::has(S - 1);
    constexpr int CB = S >= 11 ? 16 : (S == 10 ? 8 : 4);
    constexpr int NW = CB / 4;
    constexpr int PERIT = 64 * CB;
    constexpr int IT = H >= PERIT ? H / PERIT : 1;
    constexpr int U = IT < 8 ? IT : 8;
    static_assert(!(SREG || DREG) || CB == 16, "register stages use 16-byte chunks");
    const int lane = this->lane;
    const LDS unsigned char* in = this->stage(S);
    LDS unsigned char* out = this->stage(S - 1);
    if constexpr (SREG) launder<S>();
#pragma unroll
    for (int b0 = 0; b0 < IT; b0 += U) {
      uint32_t A[U][NW], Bv[U][NW], bb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = b0 + u;
        const int i0 = it * PERIT + lane * CB;
        bb[u] = 0;
        if (H >= PERIT || i0 < H) {
          if constexpr (SREG) {
#pragma unroll
            for (int k = 0; k < NW; ++k) {
              A[u][k] = rs[R::base(S) + 4 * it + k];
              Bv[u][k] = rs[R::base(S) + 4 * (it + IT) + k];
            }
          } else if constexpr (CH && CB == 16) {
            // the lane part of the offset in a register, the constant part
            // as the scalar offset (no per-iteration address registers)
            const u32x4 va =
                __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, lane * CB, it * PERIT, 0));
            const u32x4 vb = __builtin_bit_cast(
                u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, lane * CB, it * PERIT + H, 0));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              A[u][k] = va[k];
              Bv[u][k] = vb[k];
            }
          } else if constexpr (CH && CB == 8) {
            const u32x2 va =
                __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(this->chr, lane * CB, it * PERIT, 0));
            const u32x2 vb = __builtin_bit_cast(
                u32x2, __builtin_amdgcn_raw_buffer_load_b64(this->chr, lane * CB, it * PERIT + H, 0));
            A[u][0] = va[0];
            A[u][1] = va[1];
            Bv[u][0] = vb[0];
            Bv[u][1] = vb[1];
          } else if constexpr (CH) {
            A[u][0] = __builtin_amdgcn_raw_buffer_load_b32(this->chr, lane * CB, it * PERIT, 0);
            Bv[u][0] = __builtin_amdgcn_raw_buffer_load_b32(this->chr, lane * CB, it * PERIT + H, 0);
          } else if constexpr (CB == 16) {
            const u32x4 va = *(const LDS u32x4*)(in + i0);
            const u32x4 vb = *(const LDS u32x4*)(in + i0 + H);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              A[u][k] = va[k];
              Bv[u][k] = vb[k];
            }
          } else if constexpr (CB == 8) {
            const u32x2 va = *(const LDS u32x2*)(in + i0);
            const u32x2 vb = *(const LDS u32x2*)(in + i0 + H);
            A[u][0] = va[0];
            A[u][1] = va[1];
            Bv[u][0] = vb[0];
            Bv[u][1] = vb[1];
          } else {
            A[u][0] = *(const LDS uint32_t*)(in + i0);
            Bv[u][0] = *(const LDS uint32_t*)(in + i0 + H);
          }
          if constexpr (CODE == DOP_G) bb[u] = this->beta[(o + i0) >> 5] >> ((o + i0) & 31);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = b0 + u;
        const int i0 = it * PERIT + lane * CB;
        if (H >= PERIT || i0 < H) {
          uint32_t Rw[NW];
#pragma unroll
          for (int k = 0; k < NW; ++k) Rw[k] = fg_word<CODE, CH>(A[u][k], Bv[u][k], bb[u], k);
          if constexpr (DREG) {
#pragma unroll
            for (int k = 0; k < NW; ++k) rs[R::base(S - 1) + 4 * it + k] = Rw[k];
          } else if constexpr (CB == 16) {
            *(LDS u32x4*)(out + i0) = (u32x4){Rw[0], Rw[1], Rw[2], Rw[3]};
          } else if constexpr (CB == 8) {
            *(LDS u32x2*)(out + i0) = (u32x2){Rw[0], Rw[1]};
          } else {
            *(LDS uint32_t*)(out + i0) = Rw[0];
          }
        }
      }
    }
  }

  // ------------------------------------------- fused root-child ops
  // The node of stage L2N-1 at offset O (0 or 2^(L2N-1)) runs XC (f, g or
  // g_0R, eq. (1)/(2)) on its LLRs, which are the root's op YC applied to
  // the channel: alpha_v[i] = YC(c[i], c[i + 2^(L2N-1)]) with the root's
  // left-child bits (g).  Output: the register stage L2N-2.  Same integer
  // operations in the same order as the two separate ops.
  template <uint32_t XC, uint32_t YC, int O>
  __device__ __forceinline__ void fused_top() {
    constexpr int H1 = 1 << (L2N - 1), H2 = 1 << (L2N - 2);
    constexpr int IT = H2 / 1024;
    constexpr int U = 2;
    static_assert(VTOP == 1 && R::has(L2N - 2), "fused root-child op needs the virtual top stage");
    const int lane = this->lane;
#pragma unroll
    for (int b0 = 0; b0 < IT; b0 += U) {
      u32x4 c00[U], c01[U], c10[U], c11[U];
      uint32_t by0[U], by1[U], bx[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = b0 + u;
        const int i0 = it * 1024 + lane * 16;
        c00[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, lane * 16, it * 1024, 0));
        c01[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, lane * 16, it * 1024 + H1, 0));
        c10[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, lane * 16, it * 1024 + H2, 0));
        c11[u] =
            __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, lane * 16, it * 1024 + H2 + H1, 0));
        by0[u] = by1[u] = bx[u] = 0;
        if constexpr (YC == DOP_G) {  // bits of the root's left child, at i and i + H2
          by0[u] = this->beta[i0 >> 5] >> (i0 & 31);
          by1[u] = this->beta[(i0 + H2) >> 5] >> ((i0 + H2) & 31);
        }
        if constexpr (XC == DOP_G) bx[u] = this->beta[(O + i0) >> 5] >> ((O + i0) & 31);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int it = b0 + u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          // even LLRs clean, odd ones garbled; the a operands of g clean
          s2 a0e = even_lanes(c00[u][k]), a1e = even_lanes(c01[u][k]);
          s2 b0e = even_lanes(c10[u][k]), b1e = even_lanes(c11[u][k]);
          s2 a0o = odd_lanes(c00[u][k]), a1o = odd_lanes(c01[u][k]);
          s2 b0o = odd_lanes(c10[u][k]), b1o = odd_lanes(c11[u][k]);
          if constexpr (YC != DOP_F) {  // channel values feeding g
            a0o = clean(a0o), b0o = clean(b0o);
            a0e = chanx(a0e), a1e = chanx(a1e), b0e = chanx(b0e), b1e = chanx(b1e);
            a0o = chanx(a0o), a1o = chanx(a1o), b0o = chanx(b0o), b1o = chanx(b1o);
          }
          s2 xe, xo, ye, yo;
          if constexpr (YC == DOP_F) {
            xe = fx(a0e, a1e);
            xo = fx(a0o, a1o);
            ye = fx(b0e, b1e);
            yo = fx(b0o, b1o);
          } else if constexpr (YC == DOP_G) {
            const u32x2 sx = this->gsigns(by0[u], k);
            const u32x2 sy = this->gsigns(by1[u], k);
            xe = gx(a0e, a1e, as_s2(sx[0]));
            xo = gx(a0o, a1o, as_s2(sx[1]));
            ye = gx(b0e, b1e, as_s2(sy[0]));
            yo = gx(b0o, b1o, as_s2(sy[1]));
          } else {
            xe = g0x(a0e, a1e);
            xo = g0x(a0o, a1o);
            ye = g0x(b0e, b1e);
            yo = g0x(b0o, b1o);
          }
          s2 re, ro;
          if constexpr (XC == DOP_F) {
            re = fx(xe, ye);
            ro = fx(xo, yo);
          } else if constexpr (XC == DOP_G) {  // the a operand (x) clean
            const u32x2 sg = this->gsigns(bx[u], k);
            re = gx(clean(xe), ye, as_s2(sg[0]));
            ro = gx(clean(xo), yo, as_s2(sg[1]));
          } else {
            re = g0x(clean(xe), ye);
            ro = g0x(clean(xo), yo);
          }
          rs[R::base(L2N - 2) + 4 * it + k] = pack_eo(re, ro);
        }
      }
    }
  }

  // The float form of fused_top: the same two ops on float LLRs, output
  // stage L2N-2 (the float register stage when the layout has one, else
  // LDS).
  template <uint32_t XC, uint32_t YC, int O>
  __device__ __forceinline__ void fused_top_f32() {
    constexpr int H1 = 1 << (L2N - 1), H2 = 1 << (L2N - 2);
    constexpr int PERIT = 256;  // 4 floats per lane
    constexpr int IT = H2 / PERIT;
    constexpr int U = 4;
    static_assert(VTOP == 1 && NREG <= 1 && IT % U == 0, "float fused root-child op layout");
    constexpr bool DREG = R::has(L2N - 2);
    const int lane = this->lane;
    LDS float* out = (LDS float*)this->stage(L2N - 2);
#pragma unroll
    for (int b0 = 0; b0 < IT; b0 += U) {
      u32x4 c00[U], c01[U], c10[U], c11[U];
      uint32_t by0[U], by1[U], bx[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j0 = (b0 + u) * PERIT + lane * 4;
        const int sb = 4 * (b0 + u) * PERIT;  // bytes, wave-uniform
        c00[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, 16 * lane, sb, 0));
        c01[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, 16 * lane, sb + 4 * H1, 0));
        c10[u] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, 16 * lane, sb + 4 * H2, 0));
        c11[u] = __builtin_bit_cast(u32x4,
                                    __builtin_amdgcn_raw_buffer_load_b128(this->chr, 16 * lane, sb + 4 * (H2 + H1), 0));
        by0[u] = by1[u] = bx[u] = 0;
        if constexpr (YC == DOP_G) {  // bits of the root's left child, at j and j + H2
          by0[u] = this->beta[j0 >> 5] >> (j0 & 31);
          by1[u] = this->beta[(j0 + H2) >> 5] >> ((j0 + H2) & 31);
        }
        if constexpr (XC == DOP_G) bx[u] = this->beta[(O + j0) >> 5] >> ((O + j0) & 31);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j0 = (b0 + u) * PERIT + lane * 4;
        uint32_t Rv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float a0 = __uint_as_float(c00[u][k]), a1 = __uint_as_float(c01[u][k]);
          const float b0v = __uint_as_float(c10[u][k]), b1 = __uint_as_float(c11[u][k]);
          float x, y;
          if constexpr (YC == DOP_F) {
            x = fmin_sum(a0, a1);
            y = fmin_sum(b0v, b1);
          } else if constexpr (YC == DOP_G) {  // b + (-a) is exactly b - a
            x = __fadd_rn(a1, __uint_as_float(c00[u][k] ^ ((by0[u] << (31 - k)) & 0x80000000u)));
            y = __fadd_rn(b1, __uint_as_float(c10[u][k] ^ ((by1[u] << (31 - k)) & 0x80000000u)));
          } else {
            x = __fadd_rn(a1, a0);
            y = __fadd_rn(b1, b0v);
          }
          float r;
          if constexpr (XC == DOP_F)
            r = fmin_sum(x, y);
          else if constexpr (XC == DOP_G)
            r = __fadd_rn(y, __uint_as_float(__float_as_uint(x) ^ ((bx[u] << (31 - k)) & 0x80000000u)));
          else
            r = __fadd_rn(y, x);
          Rv[k] = __float_as_uint(r);
        }
        if constexpr (DREG) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            // computed here: sunk into its readers, each value would keep
            // its four channel LLRs alive instead of one register
            asm volatile("" : "+v"(Rv[k]));
            rs[R::base(L2N - 2) + 4 * (b0 + u) + k] = Rv[k];
          }
        } else {
          *(LDS u32x4*)(out + j0) = (u32x4){Rv[0], Rv[1], Rv[2], Rv[3]};
        }
      }
    }
  }

  template <uint32_t W, uint32_t YC>
  __device__ __forceinline__ void step_fused() {
    fresh_lane();
    if constexpr (P::ELEM == 1)
      fused_top<W & 0xffu, YC, (int)(W >> 16)>();
    else
      fused_top_f32<W & 0xffu, YC, (int)(W >> 16)>();
    wave_sync();
  }

  // ------------------------------------ virtual stage below the registers
  // One float f / g / g_0R as the separate ops compute it: a = alpha_v[i],
  // b = alpha_v[i + h] (bit patterns), `bits`: beta_l of LLRs i .. i+3 from
  // bit 0 (g), k: which of the four.
  template <uint32_t C>
  static __device__ __forceinline__ float op_f32(uint32_t a, uint32_t b, uint32_t bits, int k) {
    if constexpr (C == DOP_F)
      return fmin_sum(__uint_as_float(a), __uint_as_float(b));
    else if constexpr (C == DOP_G)  // b + (-a) is exactly b - a
      return __fadd_rn(__uint_as_float(b), __uint_as_float(a ^ ((bits << (31 - k)) & 0x80000000u)));
    else
      return __fadd_rn(__uint_as_float(b), __uint_as_float(a));
  }

  // f / g / g_0R (XC) of the node of stage kVMid at offset o, whose LLRs are
  // YC (the parent's op: f for a left child, g or g_0R for a right one) of
  // the register stage: alpha[j] = YC(A[j], A[j + H1]), and the output
  // XC(alpha[j], alpha[j + H2]) goes to LDS stage kVMid - 1.  Same float
  // operations in the same order as the two separate ops; every operand of
  // lane L is in lane L (a register stage holds LLRs 4L .. 4L+3 of each
  // block of 256).
  template <uint32_t XC, uint32_t YC>
  __device__ __forceinline__ void fg_mid_f32(int o) {
    constexpr int H1 = 1 << kVMid, H2 = H1 >> 1;
    constexpr int NB = H2 / 256;                     // output blocks of 256 LLRs
    constexpr int RH1 = 4 * (H1 / 256), RH2 = 4 * (H2 / 256);  // register distances of + H1, + H2
    const int lane = this->lane;
    const int op = o & ~(2 * H1 - 1);                // the parent, at the register stage
    LDS float* out = (LDS float*)this->stage(kVMid - 1);
    // beta bits of LLRs p + 4 L .. p + 4 L + 3 (p a multiple of 256): bits
    // 4 (L & 7) .. of word p / 32 + L / 8 (one lane offset for every block)
    const LDS uint32_t* bl = this->beta + (lane >> 3);
    const int sh = (lane & 7) << 2;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j0 = 256 * b + 4 * lane;
      uint32_t by0 = 0, by1 = 0, bx = 0;
      if constexpr (YC == DOP_G) {  // bits of the parent's left child at j and j + H2
        by0 = bl[(op + 256 * b) >> 5] >> sh;
        by1 = bl[(op + 256 * b + H2) >> 5] >> sh;
      }
      if constexpr (XC == DOP_G) bx = bl[(o + 256 * b) >> 5] >> sh;
      uint32_t Rv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = R::base(kVMid + 1) + 4 * b + k;
        const float x = op_f32<YC>(rs[r], rs[r + RH1], by0, k);
        const float y = op_f32<YC>(rs[r + RH2], rs[r + RH2 + RH1], by1, k);
        Rv[k] = __float_as_uint(op_f32<XC>(__float_as_uint(x), __float_as_uint(y), bx, k));
      }
      *(LDS u32x4*)(out + j0) = (u32x4){Rv[0], Rv[1], Rv[2], Rv[3]};
    }
  }

  // Rate-1 or SPC leaf of stage kVMid at offset o, its LLRs YC of the
  // register stage (as in fg_mid_f32), recomputed where they are read.
  template <uint32_t YC>
  __device__ __forceinline__ void leaf_mid_f32(uint32_t code, int o) {
    constexpr int H1 = 1 << kVMid, RH1 = 4 * (H1 / 256);
    const int op = o & ~(2 * H1 - 1);
    const LDS uint32_t* bl = this->beta + (this->lane >> 3);  // as in fg_mid_f32
    const int sh = (this->lane & 7) << 2;
    auto val = [&](int b, int k) -> float {
      uint32_t by = 0;
      if constexpr (YC == DOP_G) by = bl[(op + 256 * b) >> 5] >> sh;
      const int r = R::base(kVMid + 1) + 4 * b + k;
      return op_f32<YC>(rs[r], rs[r + RH1], by, k);
    };
    leaf_values_f32<kVMid>(code, o, val);
  }

  // With VMID the register stage leaves little room: a new name for the
  // lane index at every op keeps the compiler from computing lane-based
  // addresses once for the whole kernel and holding them (or spilling them).
  __device__ __forceinline__ void fresh_lane() {
    if constexpr (VMID) asm volatile("" : "+v"(this->lane));
  }

  template <uint32_t W, uint32_t YC>
  __device__ __forceinline__ void step_mid() {
    fresh_lane();
    constexpr uint32_t code = W & 0xffu;
    static_assert(VMID == 1 && (int)((W >> 8) & 0xffu) == kVMid, "an op of the virtual stage");
    static_assert(code <= DOP_G0R || code == DOP_R1 || code == DOP_SPC, "f, g, g_0R, Rate-1 or SPC");
    if constexpr (code <= DOP_G0R) {
      fg_mid_f32<code, YC>((int)(W >> 16));
    } else {
      leaf_mid_f32<YC>(code, (int)(W >> 16));
      this->settle();
    }
    wave_sync();
  }

  // ------------------------------------------------ wide F / G (float)
  template <int S, uint32_t CODE>
  __device__ __forceinline__ void fg_f32(int o) {
    constexpr int H = 1 << (S - 1);
    constexpr bool CH = S == L2N;
    constexpr int PERIT = 256;  // 4 floats per lane
    constexpr int IT = H >= PERIT ? H / PERIT : 1;
    constexpr int U = IT < 8 ? IT : 8;
    const int lane = this->lane;
    const LDS float* in = (const LDS float*)this->stage(S);
    LDS float* out = (LDS float*)this->stage(S - 1);
#pragma unroll
    for (int b0 = 0; b0 < IT; b0 += U) {
      u32x4 va[U], vb[U];
      uint32_t bb[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i0 = (b0 + u) * PERIT + lane * 4;
        bb[u] = 0;
        if (H >= PERIT || i0 < H) {
          if constexpr (R::has(S)) {  // block it and it + IT of this lane
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              va[u][k] = rs[R::base(S) + 4 * (b0 + u) + k];
              vb[u][k] = rs[R::base(S) + 4 * (b0 + u + IT) + k];
            }
          } else if constexpr (CH) {
            va[u] = __builtin_bit_cast(
                u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, 16 * lane, 4 * (b0 + u) * PERIT, 0));
            vb[u] = __builtin_bit_cast(
                u32x4, __builtin_amdgcn_raw_buffer_load_b128(this->chr, 16 * lane, 4 * ((b0 + u) * PERIT + H), 0));
          } else {
            va[u] = *(const LDS u32x4*)(in + i0);
            vb[u] = *(const LDS u32x4*)(in + i0 + H);
          }
          if constexpr (CODE == DOP_G) bb[u] = this->beta[(o + i0) >> 5] >> ((o + i0) & 31);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i0 = (b0 + u) * PERIT + lane * 4;
        if (H >= PERIT || i0 < H) {
          float Rv[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float a = __uint_as_float(va[u][k]), b = __uint_as_float(vb[u][k]);
            if constexpr (CODE == DOP_F)
              Rv[k] = fmin_sum(a, b);
            else if constexpr (CODE == DOP_G)  // b + (-a) is exactly b - a
              Rv[k] = __fadd_rn(b, __uint_as_float(va[u][k] ^ ((bb[u] << (31 - k)) & 0x80000000u)));
            else
              Rv[k] = __fadd_rn(b, a);
          }
          *(LDS u32x4*)(out + i0) = (u32x4){__float_as_uint(Rv[0]), __float_as_uint(Rv[1]), __float_as_uint(Rv[2]),
                                            __float_as_uint(Rv[3])};
        }
      }
    }
  }

  // ------------------------------------------ leaves at register stages
  // 16 hard decisions of lane chunk `it` of register stage S.
  template <int S>
  __device__ __forceinline__ uint32_t reg_hd16(int it) const {
    uint32_t d = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      d |= __builtin_amdgcn_udot4((rs[R::base(S) + 4 * it + k] >> 7) & 0x01010101u, 0x08040201u, 0u, false)
           << (4 * k);
    return d;
  }

  template <int S>
  __device__ __forceinline__ int reg_elem(int it, int k, int b) const {
    const int x = (int)(int8_t)(rs[R::base(S) + 4 * it + k] >> (8 * b));
    return x < -127 ? -127 : x;
  }

  // Rate-1, repetition or SPC leaf whose LLRs are a register stage S.
  template <int S>
  __device__ __forceinline__ void leaf_reg(uint32_t code, int o) {
    constexpr int NV = 1 << S;
    constexpr int IT = NV >> 10;
    constexpr int NW = NV >> 5;
    constexpr int PER = NW / 64;
    const int lane = this->lane;
    LDS uint32_t* bw = this->beta + (o >> 5);
    launder<S>();
    if (this->tr) {
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            this->tr[o + 1024 * it + 16 * lane + 4 * k + b] = (int8_t)reg_elem<S>(it, k, b);
    }
    if (code == DOP_REP) {
      // integers: every partial sum is exact, so the order is free
      int sum = 0;
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int b = 0; b < 4; ++b) sum += reg_elem<S>(it, k, b);
      float sf = (float)sum;
      sf += __shfl_xor(sf, 32, 64);
      sf += __shfl_xor(sf, 16, 64);
      sf += __shfl_xor(sf, 8, 64);
      sf += __shfl_xor(sf, 4, 64);
      sf += __shfl_xor(sf, 2, 64);
      sf += __shfl_xor(sf, 1, 64);
      const bool bit = rflf(sf) < 0.0f;
      for (int j = lane; j < NW; j += 64) bw[j] = bit ? ~0u : 0u;
      this->pend_v = bit ? 1ull : 0ull;
      this->pend_n = 1;
      return;
    }
    // beta words to LDS: word 32 it + L/2 is the chunks of lanes L, L+1
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const uint32_t c = reg_hd16<S>(it);
      const uint32_t up = from_up<1>(c);
      if ((lane & 1) == 0) bw[32 * it + (lane >> 1)] = c | (up << 16);
    }
    wave_sync();
    uint32_t wd[PER];
    int par = 0;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      wd[m] = bw[lane + 64 * m];
      par ^= __popc(wd[m]);
    }
    if (code == DOP_SPC && (__popcll(ballot((par & 1) != 0)) & 1)) {
      float best = 3.0e38f;
      int bi = 0x7fffffff;
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int x = reg_elem<S>(it, k, b);
            const float m = (float)(x < 0 ? -x : x);
            if (m < best) {  // this lane's indices grow in this order
              best = m;
              bi = 1024 * it + 16 * lane + 4 * k + b;
            }
          }
      const int idx = this->argmin_reduce(best, bi);
      const int jw = idx >> 5;
      if ((jw & 63) == lane) {
#pragma unroll
        for (int m = 0; m < PER; ++m)
          if (m == (jw >> 6)) {
            wd[m] ^= 1u << (idx & 31);
            bw[jw] = wd[m];
          }
      }
    }
    this->template finish_leaf<S, PER>(wd, code, (LDS uint32_t*)this->stage(kTopLds));
  }

  // Rate-1, repetition or SPC leaf whose float LLRs are a register stage S
  // (LLR e in lane (e >> 2) & 63, register 4 (e >> 8) + (e & 3)).
  template <int S>
  __device__ __forceinline__ void leaf_reg_f32(uint32_t code, int o) {
    constexpr int NV = 1 << S;
    constexpr int NB = NV >> 8;  // blocks of 256 LLRs, 4 registers each
    constexpr int NW = NV >> 5;
    const int lane = this->lane;
    LDS uint32_t* bw = this->beta + (o >> 5);
    if (code == DOP_REP) {
      if (this->tr) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int k = 0; k < 4; ++k) this->tr[o + 256 * b + 4 * lane + k] = __uint_as_float(rs[R::base(S) + 4 * b + k]);
      }
      // the halving tree s_i <- s_i + s_{i+d}, d = NV/2 .. 1, one rounded add each
      float v[4 * NB];
#pragma unroll
      for (int r = 0; r < 4 * NB; ++r) v[r] = __uint_as_float(rs[R::base(S) + r]);
#pragma unroll
      for (int nb = NB / 2; nb >= 1; nb /= 2)  // d = 256 nb: register r + 4 nb of the same lane
#pragma unroll
        for (int r = 0; r < 4 * nb; ++r) v[r] = __fadd_rn(v[r], v[r + 4 * nb]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {  // d = 128 .. 4: lane + d / 4
        v[k] = __fadd_rn(v[k], from_up<32>(v[k]));
        v[k] = __fadd_rn(v[k], from_up<16>(v[k]));
        v[k] = __fadd_rn(v[k], from_up<8>(v[k]));
        v[k] = __fadd_rn(v[k], from_up<4>(v[k]));
        v[k] = __fadd_rn(v[k], from_up<2>(v[k]));
        v[k] = __fadd_rn(v[k], from_up<1>(v[k]));
      }
      v[0] = __fadd_rn(v[0], v[2]);  // d = 2, 1: in lane 0
      v[1] = __fadd_rn(v[1], v[3]);
      v[0] = __fadd_rn(v[0], v[1]);
      const bool bit = rflf(v[0]) < 0.0f;
      for (int j = lane; j < NW; j += 64) bw[j] = bit ? ~0u : 0u;
      this->pend_v = bit ? 1ull : 0ull;
      this->pend_n = 1;
      return;
    }
    leaf_values_f32<S>(code, o, [&](int b, int k) { return __uint_as_float(rs[R::base(S) + 4 * b + k]); });
  }

  // Rate-1 or SPC leaf of 2^S float LLRs in the register-stage order: val(b,
  // k) is LLR 256 b + 4 L + k of lane L (read as often as needed).
  template <int S, class V>
  __device__ __forceinline__ void leaf_values_f32(uint32_t code, int o, const V& val) {
    constexpr int NV = 1 << S;
    constexpr int NB = NV >> 8;  // blocks of 256 LLRs
    constexpr int NW = NV >> 5;
    constexpr int PER = NW / 64;
    static_assert(PER >= 1, "a float register-order leaf holds >= 2048 LLRs");
    const int lane = this->lane;
    LDS uint32_t* bw = this->beta + (o >> 5);
    if (this->tr) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k) this->tr[o + 256 * b + 4 * lane + k] = val(b, k);
    }
    // beta words to LDS: in block b, lane L holds the hard decisions of LLRs
    // 4L .. 4L+3, a nibble of word 8b + L/8
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      uint32_t nib = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) nib |= (val(b, k) < 0.0f ? 1u : 0u) << k;
      uint32_t t = nib << (4 * (lane & 7));
      t |= from_up<4>(t);
      t |= from_up<2>(t);
      t |= from_up<1>(t);
      if ((lane & 7) == 0) bw[8 * b + (lane >> 3)] = t;
    }
    wave_sync();
    uint32_t wd[PER];
    int par = 0;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      wd[m] = bw[lane + 64 * m];
      par ^= __popc(wd[m]);
    }
    if (code == DOP_SPC && (__popcll(ballot((par & 1) != 0)) & 1)) {
      float best = 3.0e38f;
      int bi = 0x7fffffff;
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float m = fabsf(val(b, k));
          if (m < best) {  // this lane's indices grow in this order
            best = m;
            bi = 256 * b + 4 * lane + k;
          }
        }
      const int idx = this->argmin_reduce(best, bi);
      const int jw = idx >> 5;
      if ((jw & 63) == lane) {
#pragma unroll
        for (int m = 0; m < PER; ++m)
          if (m == (jw >> 6)) {
            wd[m] ^= 1u << (idx & 31);
            bw[jw] = wd[m];
          }
      }
    }
    this->template finish_leaf<S, PER>(wd, code, (LDS uint32_t*)this->stage(kTopLds));
  }

  // ----------------------------------------------------------- one op
  template <uint32_t W>
  __device__ __forceinline__ void step_c() {
    fresh_lane();
    constexpr uint32_t code = W & 0xffu;
    constexpr int S = (int)((W >> 8) & 0xffu);
    constexpr int o = (int)(W >> 16);
    if constexpr (S <= kRegStages) {
      if constexpr (code <= DOP_G0R)
        this->template small_fg<S>(code, o);
      else if constexpr (code <= DOP_CR0)
        this->small_combine(code, S, o);
      else if constexpr (code == DOP_FLUSH)
        this->flush(o);
      else if constexpr (is_pair_op(code))
        this->template small_pair<S>(code, o);
      else
        this->template small_leaf<S>(code, o);
    } else if constexpr (code <= DOP_G0R) {
      if constexpr (S == 7)
        this->fg7(code);
      else if constexpr (P::ELEM == 1)
        fg_i8<S, code>(o);
      else
        fg_f32<S, code>(o);
    } else if constexpr (code <= DOP_CR0) {
      this->big_combine(code, S, o);
    } else if constexpr (R::has(S)) {
      if constexpr (P::ELEM == 1)
        leaf_reg<S>(code, o);
      else
        leaf_reg_f32<S>(code, o);
    } else if constexpr (code == DOP_REP) {
      this->big_leaf(code, S, o);
    } else {
      this->template leaf_r1spc<S>(code, o, S - 1 < kTopLds ? S - 1 : kTopLds);
    }
    if constexpr ((code >= DOP_R1 && code <= DOP_SPC) || is_pair_op(code)) this->settle();
    // Ops on nodes of size <= 64 touch only registers and the output row
    // (FLUSH aside), so consecutive ones need no ordering point and the
    // compiler may interleave them.
    if constexpr (S > kRegStages || code == DOP_FLUSH) wave_sync();
  }
};

}  // namespace
}  // namespace polar
