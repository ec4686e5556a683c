// Device codec for the reduced storage formats (Sec. IV-A: ExMy formats packed several to a 32-bit
// word; Sec. V-B: FP32 -> narrow on write, narrow -> FP32 on read, arithmetic in FP32).
//
// Encoding rounds to nearest with ties to even and keeps subnormals.  FP16/BF16 overflow to Inf;
// E4M3/E5M2/E3M2/E2M1 saturate to their largest finite magnitude (Inf inputs too).  NaN inputs give
// the format's quiet NaN where it has one, the largest magnitude otherwise (outside the contract).
// The encoder works on the integer fields of the FP32 input: the significand is shifted right by
// the number of bits the target cannot hold (more for targets' subnormals) with round-half-even on
// the dropped bits, and the rounded significand is added to the target exponent field so that a
// carry moves to the next binade by itself.  Decoding places the code's exponent/mantissa fields at
// the top of an FP32 word and rescales by a power of two, which is exact for normal and subnormal
// codes alike.
//
// Packed groups: N values of b bits form a little-endian bit stream of ceil(N*b/32) dwords, value i
// at bits [b*i, b*i+b).  The scalar integer encoder/decoder define the conversions; the group
// codec used by the kernels runs on the native conversion instructions, which match them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vapr {

// PXM: an emulated ExMy type stored as its own packed codes (E and M travel beside the format id)
enum : int { F32 = 0, F16 = 1, BF16 = 2, E4M3 = 3, E5M2 = 4, E3M2 = 5, E2M1 = 6, PXM = 7, N_FORMATS = 8 };

template <int F> struct Fmt;
//                 E   M  bias sat   bits  max magnitude  inf       nan
template <> struct Fmt<F16>  { static constexpr int E = 5, M = 10, BIAS = 15,  BITS = 16; static constexpr bool SAT = false; static constexpr uint32_t MAXMAG = 0x7BFF, INF = 0x7C00, QNAN = 0x7E00; };
template <> struct Fmt<BF16> { static constexpr int E = 8, M = 7,  BIAS = 127, BITS = 16; static constexpr bool SAT = false; static constexpr uint32_t MAXMAG = 0x7F7F, INF = 0x7F80, QNAN = 0x7FC0; };
template <> struct Fmt<E4M3> { static constexpr int E = 4, M = 3,  BIAS = 7,   BITS = 8;  static constexpr bool SAT = true;  static constexpr uint32_t MAXMAG = 0x7E,   INF = 0x7E,   QNAN = 0x7F; };
template <> struct Fmt<E5M2> { static constexpr int E = 5, M = 2,  BIAS = 15,  BITS = 8;  static constexpr bool SAT = true;  static constexpr uint32_t MAXMAG = 0x7B,   INF = 0x7B,   QNAN = 0x7E; };
template <> struct Fmt<E3M2> { static constexpr int E = 3, M = 2,  BIAS = 3,   BITS = 6;  static constexpr bool SAT = true;  static constexpr uint32_t MAXMAG = 0x1F,   INF = 0x1F,   QNAN = 0x1F; };
template <> struct Fmt<E2M1> { static constexpr int E = 2, M = 1,  BIAS = 1,   BITS = 4;  static constexpr bool SAT = true;  static constexpr uint32_t MAXMAG = 0x7,    INF = 0x7,    QNAN = 0x7; };
template <> struct Fmt<F32>  { static constexpr int E = 8, M = 23, BIAS = 127, BITS = 32; static constexpr bool SAT = false; static constexpr uint32_t MAXMAG = 0x7F7FFFFF, INF = 0x7F800000, QNAN = 0x7FC00000; };

__host__ __device__ constexpr int format_bits(int f) {
  return f == F32 ? 32 : (f == F16 || f == BF16) ? 16 : (f == E4M3 || f == E5M2) ? 8 : f == E3M2 ? 6 : 4;
}
// dwords holding a packed group of n values
__host__ __device__ constexpr int group_dwords(int f, int n) { return (format_bits(f) * n + 31) / 32; }

// ---- generic ExMy rounding (emulated formats) --------------------------------------------------
//
// The nearest value of the type with E exponent and M mantissa bits (bias 2^(E-1) - 1, subnormals
// kept), ties to even: the grid spacing at |y| = m 2^e is 2^(max(e, e_min) - M), and |y| is scaled
// to it, rounded to an integer and scaled back (each step exact in FP32 for E <= 8, M <= 23).
// E5M10 and the types with 8 exponent bits follow IEEE (top exponent field reserved, rounding past
// the largest finite value gives Inf; without the reserved field an 8-bit exponent would reach
// 2^128, beyond FP32); every other type is finite-only and saturates, Inf inputs included.  Zero and
// NaN pass through.
__device__ __forceinline__ float exmy_round(float y, int E, int M) {
  const float a = fabsf(y);
  if (!(a > 0.f)) return y;
  const int bias = (1 << (E - 1)) - 1;
  const int e_min = 1 - bias;
  const bool ieee = (E == 5 && M == 10) || E == 8;
  const int e_max = (ieee ? (1 << E) - 2 : (1 << E) - 1) - bias;
  const float vmax = ldexpf(2.f - ldexpf(1.f, -M), e_max);
  float r;
  if (a == INFINITY) {
    r = ieee ? INFINITY : vmax;
  } else {
    const int eb = (int)((__float_as_uint(a) >> 23) & 0xffu);
    const int e = eb ? eb - 127 : -127;
    const int q = (e > e_min ? e : e_min) - M;
    r = ldexpf(rintf(ldexpf(a, -q)), q);
    if (r > vmax) r = ieee ? INFINITY : vmax;
  }
  return copysignf(r, y);
}

// ---- packed ExMy codes (emulated types stored in their own bits) --------------------------------
//
// Code of a value of the type: sign at bit E + M, the biased exponent field (0 for zero and
// subnormals), M mantissa bits.  A 32-bit word holds q = floor(32 / b) codes, b = 1 + E + M, from the
// low bits up (one FP32, two FP16, three FP10, four FP8, five FP6, six FP5 or eight FP4 a register,
// Sec. IV-A); the top 32 - q b bits stay zero.  A group of n values takes ceil(n / q) words.

__host__ __device__ constexpr int pxm_per_word(int E, int M) { return 32 / (1 + E + M); }
__host__ __device__ constexpr int pxm_group_dwords(int E, int M, int n) {
  return (n + pxm_per_word(E, M) - 1) / pxm_per_word(E, M);
}

// The code of exmy_round(y): the rounded value is representable, so its fields are read off its FP32
// bits -- exponent rebiased and mantissa truncated to M bits for normal values, the significand
// shifted to the subnormal grid 2^(e_min - M) otherwise.  Inf gives the Inf code and NaN the quiet
// NaN of the IEEE-like types; a NaN of the saturating types (outside the contract) stores the
// largest magnitude.
__device__ __forceinline__ uint32_t exmy_encode(float y, int E, int M) {
  const uint32_t u = __float_as_uint(exmy_round(y, E, M));
  const uint32_t sign = (u >> 31) << (E + M);
  const uint32_t a = u & 0x7fffffffu;
  const uint32_t top = (1u << E) - 1u;
  if (a >= 0x7f800000u) {
    const bool ieee = (E == 5 && M == 10) || E == 8;
    if (ieee) return sign | (top << M) | (a > 0x7f800000u && M > 0 ? 1u << (M - 1) : 0u);
    return sign | (top << M) | ((1u << M) - 1u);
  }
  if (a == 0u) return sign;
  const int bias = (1 << (E - 1)) - 1;
  const int e_min = 1 - bias;
  const int fe = (int)(a >> 23);
  if (fe != 0 && fe - 127 >= e_min) return sign | ((uint32_t)(fe - 127 + bias) << M) | ((a & 0x7fffffu) >> (23 - M));
  const uint32_t sig = (a & 0x7fffffu) | (fe ? 0x800000u : 0u);  // value = sig 2^(max(fe, 1) - 150)
  const int sh = (e_min - M) - ((fe ? fe : 1) - 150);
  return sign | (sh >= 32 ? 0u : sig >> sh);
}

__device__ __forceinline__ float exmy_decode(uint32_t c, int E, int M) {
  const uint32_t mag = c & ((1u << (E + M)) - 1u);
  const uint32_t ef = mag >> M, mant = mag & ((1u << M) - 1u);
  const int bias = (1 << (E - 1)) - 1;
  const bool ieee = (E == 5 && M == 10) || E == 8;
  float v;
  if (ieee && ef == (1u << E) - 1u) v = mant ? __uint_as_float(0x7fc00000u) : __uint_as_float(0x7f800000u);
  else if (ef == 0u) v = ldexpf((float)mant, 1 - bias - M);
  else v = ldexpf((float)((1u << M) | mant), (int)ef - bias - M);
  return ((c >> (E + M)) & 1u) ? -v : v;
}

// a group of N values as ceil(N / Q) words (Q = codes per word)
// Group of N values to packed codes: q = floor(32 / b) codes per word, code i at bits (i % q) b of
// word i / q, written to base[k * stride] for word k.  q is a runtime property of the type; the walk
// keeps one word in flight, so the code does not depend on q.
template <int N>
__device__ __forceinline__ void pxm_store_words(const float (&v)[N], int E, int M, int q, float inv, uint32_t* base,
                                                int stride) {
  const int b = 1 + E + M;
  uint32_t acc = 0u;
  int c = 0, k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    acc |= exmy_encode(v[i] * inv, E, M) << (c * b);
    if (++c == q) {
      base[k * stride] = acc;
      ++k;
      acc = 0u;
      c = 0;
    }
  }
  if (c) base[k * stride] = acc;
}

template <int N>
__device__ __forceinline__ void pxm_load_words(const uint32_t* base, int stride, int E, int M, int q, float scale,
                                               float (&v)[N]) {
  const int b = 1 + E + M;
  const uint32_t mask = b >= 32 ? 0xffffffffu : (1u << b) - 1u;
  uint32_t w = base[0];
  int c = 0, k = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (c == q) {
      w = base[++k * stride];
      c = 0;
    }
    v[i] = exmy_decode((w >> (c * b)) & mask, E, M) * scale;
    ++c;
  }
}

// ---- scalar encode / decode -------------------------------------------------------------------

template <int F>
__device__ __forceinline__ uint32_t encode(float y) {
  using T = Fmt<F>;
  const uint32_t u = __float_as_uint(y);
  if constexpr (F == F32) {
    return u;
  } else {
    const uint32_t sign = (u >> 31) << (T::E + T::M);
    const uint32_t a = u & 0x7fffffffu;
    if (a >= 0x7f800000u) {  // Inf or NaN
      if (a == 0x7f800000u) return sign | T::INF;
      return sign | T::QNAN;
    }
    const int e = (int)(a >> 23);
    const uint32_t sig = (a & 0x7fffffu) | (e ? 0x800000u : 0u);
    const int ee = e ? e : 1;                 // FP32 subnormals share the exponent of e = 1
    const int et = ee - 127 + T::BIAS;        // target biased exponent if the result is normal
    int shift = 23 - T::M + (et < 1 ? 1 - et : 0);
    shift = shift > 25 ? 25 : shift;          // sig < 2^24: at 25 everything rounds to zero
    uint32_t q = sig >> shift;
    const uint32_t rem = sig & ((1u << shift) - 1u);
    const uint32_t half = 1u << (shift - 1);
    q += (rem > half) | ((rem == half) & (q & 1u));
    const uint32_t base = et < 1 ? 0u : (uint32_t)(et - 1);
    uint32_t mag = (base << T::M) + q;        // rounded significand carries into the exponent
    if (mag > T::MAXMAG) mag = T::INF;        // INF == MAXMAG for saturating formats
    return sign | mag;
  }
}

template <int F>
__device__ __forceinline__ float decode(uint32_t c) {
  using T = Fmt<F>;
  if constexpr (F == F32) {
    return __uint_as_float(c);
  } else {
    constexpr uint32_t MAGMASK = (1u << (T::E + T::M)) - 1u;
    const uint32_t mag = c & MAGMASK;
    const uint32_t sign = (c >> (T::E + T::M)) << 31;
    float v;
    if constexpr (F == BF16) {
      v = __uint_as_float(mag << 16);       // BF16 is the top half of an FP32
    } else {
      // fields at the top of an FP32 word: value * 2^(BIAS-127); rescale (exact)
      constexpr float RESCALE = __builtin_bit_cast(float, (uint32_t)(254 - T::BIAS) << 23);
      v = __uint_as_float(mag << (23 - T::M)) * RESCALE;
      if constexpr (F == F16 || F == E5M2) {
        if ((mag >> T::M) == (1u << T::E) - 1u)
          v = (mag & ((1u << T::M) - 1u)) ? __uint_as_float(0x7fc00000u) : __uint_as_float(0x7f800000u);
      }
      if constexpr (F == E4M3) {
        if (mag == 0x7Fu) v = __uint_as_float(0x7fc00000u);
      }
    }
    return __uint_as_float(__float_as_uint(v) | sign);
  }
}

// ---- group pack / unpack ----------------------------------------------------------------------

template <int F, int N>
__device__ __forceinline__ void pack_codes(const uint32_t (&c)[N], uint32_t (&w)[group_dwords(F, N)]) {
  constexpr int B = Fmt<F>::BITS;
  uint64_t acc = 0;
  int nb = 0, wi = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    acc |= (uint64_t)c[i] << nb;
    nb += B;
    if (nb >= 32) {
      w[wi++] = (uint32_t)acc;
      acc >>= 32;
      nb -= 32;
    }
  }
  if (nb > 0) w[wi++] = (uint32_t)acc;
}

template <int F, int N>
__device__ __forceinline__ void unpack_codes(const uint32_t (&w)[group_dwords(F, N)], uint32_t (&c)[N]) {
  constexpr int B = Fmt<F>::BITS;
  constexpr uint32_t MASK = B == 32 ? 0xffffffffu : ((1u << B) - 1u);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int bit = i * B, wi = bit >> 5, sh = bit & 31;
    uint64_t v = w[wi];
    if (sh + B > 32) v |= (uint64_t)w[wi + 1] << 32;
    c[i] = (uint32_t)(v >> sh) & MASK;
  }
}

// ---- group codec on the gfx950 conversion instructions ----------------------------------------
// Each native conversion below was checked against the integer encoder above on all 2^32 inputs
// and on every code: FP16/BF16 round-to-nearest-even converts, FP8 converts after clamping to the
// largest finite value (NaN passed through, because the clamp would turn it into a number), and the
// FP4/FP6 converts with unit scale.  The instructions place their first source in the lowest bits,
// which is the little-endian bit-stream layout used for packed groups.

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef uint32_t u32x6 __attribute__((ext_vector_type(6)));

template <int F>
__device__ __forceinline__ float fp8_clamp(float y) {
  constexpr float M = F == E4M3 ? 448.f : 57344.f;
  const float c = __builtin_amdgcn_fmed3f(y, -M, M);
  return y != y ? y : c;
}

template <int F, bool HI>
__device__ __forceinline__ uint32_t fp8_pack2(float a, float b, uint32_t old) {
  if constexpr (F == E4M3)
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(fp8_clamp<F>(a), fp8_clamp<F>(b), (int)old, HI);
  else
    return (uint32_t)__builtin_amdgcn_cvt_pk_bf8_f32(fp8_clamp<F>(a), fp8_clamp<F>(b), (int)old, HI);
}

template <int F, bool HI>
__device__ __forceinline__ void fp8_unpack2(uint32_t w, float& a, float& b) {
  if constexpr (F == E4M3) {
    const auto p = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, HI);
    a = p[0];
    b = p[1];
  } else {
    const auto p = __builtin_amdgcn_cvt_pk_f32_bf8((int)w, HI);
    a = p[0];
    b = p[1];
  }
}

template <int BYTE>
__device__ __forceinline__ void fp4_unpack2(uint32_t w, float& a, float& b) {
  const auto p = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(w, 1.0f, BYTE);
  a = p[0];
  b = p[1];
}

// The FP6 converts read their multi-register sources over several cycles while writing the
// result: the result registers must not overlap the sources (the early-clobber "=&v" below), which
// the compiler does not otherwise guarantee for these instructions.  The 2x16 packer interleaves
// its two sources; the 32-wide unpacker returns the codes in stream order.
__device__ __forceinline__ u32x6 fp6_pack32(f32x16 a, f32x16 b) {
  u32x6 o;
  asm volatile("v_cvt_scalef32_2xpk16_bf6_f32 %0, %1, %2, 1.0" : "=&v"(o) : "v"(a), "v"(b));
  return o;
}

__device__ __forceinline__ f32x32 fp6_unpack32(u32x6 w) {
  f32x32 o;
  asm volatile("v_cvt_scalef32_pk32_f32_bf6 %0, %1, 1.0" : "=&v"(o) : "v"(w));
  return o;
}

// encode N values (scaled by inv = 2^-k first) and pack them
template <int F, int N>
__device__ __forceinline__ void encode_group(const float (&v)[N], float inv, uint32_t (&w)[group_dwords(F, N)]) {
  if constexpr (F == F32) {
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = __float_as_uint(v[i]);
  } else if constexpr (F == F16) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      // The empty asm keeps the scaled value an FP32 register: fused into v_fma_mixlo_f16 (which
      // adds +0) a product of -0 would come out as +0.
      float ya = v[2 * i] * inv, yb = v[2 * i + 1] * inv;
      asm volatile("" : "+v"(ya), "+v"(yb));
      const _Float16 a = (_Float16)ya, b = (_Float16)yb;
      w[i] = (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
  } else if constexpr (F == BF16) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      const __bf16 a = (__bf16)(v[2 * i] * inv), b = (__bf16)(v[2 * i + 1] * inv);
      w[i] = (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
  } else if constexpr (F == E4M3 || F == E5M2) {
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const uint32_t t = fp8_pack2<F, false>(v[4 * i] * inv, v[4 * i + 1] * inv, 0u);
      w[i] = fp8_pack2<F, true>(v[4 * i + 2] * inv, v[4 * i + 3] * inv, t);
    }
  } else if constexpr (F == E2M1) {
    static_assert(N % 8 == 0, "FP4 groups hold whole dwords");
#pragma unroll
    for (int i = 0; i < N / 8; ++i) {
      uint32_t t = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(0u, v[8 * i] * inv, v[8 * i + 1] * inv, 1.0f, 0);
      t = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(t, v[8 * i + 2] * inv, v[8 * i + 3] * inv, 1.0f, 1);
      t = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(t, v[8 * i + 4] * inv, v[8 * i + 5] * inv, 1.0f, 2);
      w[i] = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(t, v[8 * i + 6] * inv, v[8 * i + 7] * inv, 1.0f, 3);
    }
  } else {  // E3M2: 16 values -> 3 dwords
    static_assert(N % 16 == 0 || N == 8, "FP6 groups are 8 or a multiple of 16 values");
    constexpr int NB = (N + 15) / 16;
#pragma unroll
    for (int g = 0; g < NB; ++g) {
      // the packer interleaves its sources (output slot 2i <- a[i], 2i+1 <- b[i]): even values go
      // to a, odd values to b, and the upper 16 slots stay zero
      f32x16 a = {}, b = {};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a[i] = (g * 16 + 2 * i < N) ? v[g * 16 + 2 * i] * inv : 0.f;
        b[i] = (g * 16 + 2 * i + 1 < N) ? v[g * 16 + 2 * i + 1] * inv : 0.f;
      }
      const u32x6 o = fp6_pack32(a, b);
      if constexpr (N == 8) {
        w[0] = o[0];
        w[1] = o[1];
      } else {
        w[3 * g + 0] = o[0];
        w[3 * g + 1] = o[1];
        w[3 * g + 2] = o[2];
      }
    }
  }
}

// unpack and decode N values, scaled by scale = 2^k
template <int F, int N>
__device__ __forceinline__ void decode_group(const uint32_t (&w)[group_dwords(F, N)], float scale, float (&v)[N]) {
  if constexpr (F == F32) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = __uint_as_float(w[i]);
    return;
  } else if constexpr (F == F16) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      v[2 * i] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[i] & 0xffffu));
      v[2 * i + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[i] >> 16));
    }
  } else if constexpr (F == BF16) {
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      v[2 * i] = __uint_as_float(w[i] << 16);
      v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  } else if constexpr (F == E4M3 || F == E5M2) {
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      fp8_unpack2<F, false>(w[i], v[4 * i], v[4 * i + 1]);
      fp8_unpack2<F, true>(w[i], v[4 * i + 2], v[4 * i + 3]);
    }
  } else if constexpr (F == E2M1) {
#pragma unroll
    for (int i = 0; i < N / 8; ++i) {
      fp4_unpack2<0>(w[i], v[8 * i], v[8 * i + 1]);
      fp4_unpack2<1>(w[i], v[8 * i + 2], v[8 * i + 3]);
      fp4_unpack2<2>(w[i], v[8 * i + 4], v[8 * i + 5]);
      fp4_unpack2<3>(w[i], v[8 * i + 6], v[8 * i + 7]);
    }
  } else {  // E3M2
    constexpr int NB = (N + 15) / 16;
#pragma unroll
    for (int g = 0; g < NB; ++g) {
      u32x6 in = {0u, 0u, 0u, 0u, 0u, 0u};
      if constexpr (N == 8) {
        in[0] = w[0];
        in[1] = w[1];
      } else {
        in[0] = w[3 * g];
        in[1] = w[3 * g + 1];
        in[2] = w[3 * g + 2];
      }
      const f32x32 o = fp6_unpack32(in);
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (g * 16 + i < N) v[g * 16 + i] = o[i];
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] *= scale;
}

// value of one code (already extracted from its group), scaled
template <int F>
__device__ __forceinline__ float decode_one(uint32_t code, float scale) {
  if constexpr (F == F32) return __uint_as_float(code);
  else if constexpr (F == F16) return (float)__builtin_bit_cast(_Float16, (uint16_t)code) * scale;
  else if constexpr (F == BF16) return __uint_as_float(code << 16) * scale;
  else if constexpr (F == E4M3) return __builtin_amdgcn_cvt_f32_fp8((int)code, 0) * scale;
  else if constexpr (F == E5M2) return __builtin_amdgcn_cvt_f32_bf8((int)code, 0) * scale;
  else if constexpr (F == E2M1) return __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(code, 1.0f, 0)[0] * scale;
  else return decode<F>(code) * scale;
}

}  // namespace vapr
