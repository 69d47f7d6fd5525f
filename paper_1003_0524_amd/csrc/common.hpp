// Shared device-side definitions for the gfx950 exchange kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exc {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u4_t __attribute__((ext_vector_type(4)));

// Product modes (values match exc_precision in include/exchange.h).
enum Mode { M_F64 = 0, M_F32 = 1, M_BF16X3 = 2, M_BF16X6 = 3 };

// ---------------------------------------------------------------------------
// Per-mode traits
//   acc_t   : MFMA accumulator element (double for FP64, float otherwise)
//   lds_t   : storage of one piece of one real value in LDS / in the prepared
//             Coulomb factor (double, float, or a bf16 bit pattern)
//   NPIECE  : pieces per real value (1, 1, 2, 3)
//   KS      : k extent of one MFMA (4 for the 16x16x4 f64/f32 forms, 32 for
//             the 16x16x32 bf16 form); each lane supplies KS/4 consecutive k
// ---------------------------------------------------------------------------
template <int MODE> struct Traits;
template <> struct Traits<M_F64> {
  using acc_t = double; using lds_t = double; using accv_t = d4_t;
  static constexpr int NPIECE = 1, KS = 4, NPROD = 1;
};
template <> struct Traits<M_F32> {
  using acc_t = float; using lds_t = float; using accv_t = f4_t;
  static constexpr int NPIECE = 1, KS = 4, NPROD = 1;
};
template <> struct Traits<M_BF16X3> {
  using acc_t = float; using lds_t = uint16_t; using accv_t = f4_t;
  static constexpr int NPIECE = 2, KS = 32, NPROD = 3;
};
template <> struct Traits<M_BF16X6> {
  using acc_t = float; using lds_t = uint16_t; using accv_t = f4_t;
  static constexpr int NPIECE = 3, KS = 32, NPROD = 6;
};

// Piece pairs (a-piece, b-piece) of the split products, leading terms first:
// x2: hh, hl, lh    x3: hh, hm, mh, hl, mm, lh
__device__ __host__ constexpr int prod_a(int nsplit, int p) {
  return nsplit == 2 ? (p == 2 ? 1 : 0) : (p <= 1 ? 0 : (p == 2 ? 1 : (p == 3 ? 0 : (p == 4 ? 1 : 2))));
}
__device__ __host__ constexpr int prod_b(int nsplit, int p) {
  return nsplit == 2 ? (p == 1 ? 1 : 0) : (p == 0 ? 0 : (p == 1 ? 1 : (p == 2 ? 0 : (p == 3 ? 2 : (p == 4 ? 1 : 0)))));
}

// ---------------------------------------------------------------------------
// bf16 helpers (round to nearest even). Inputs are finite.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Split a value into NPIECE bf16 pieces, each the RNE bf16 of the remaining
// residual (the residual of a float after removing its leading bf16 is exact).
template <int NPIECE>
__device__ __forceinline__ void split_f(float x, uint16_t* out) {
  float r = x;
#pragma unroll
  for (int p = 0; p < NPIECE; ++p) {
    uint16_t h = f2bf(r);
    out[p] = h;
    r = r - bf2f(h);
  }
}
template <int NPIECE>
__device__ __forceinline__ void split_d(double x, uint16_t* out) {
  double r = x;
#pragma unroll
  for (int p = 0; p < NPIECE; ++p) {
    uint16_t h = f2bf((float)r);
    out[p] = h;
    r = r - (double)bf2f(h);
  }
}

// Store one real value into its NPIECE LDS/global planes (plane stride `ps`).
template <int MODE>
__device__ __forceinline__ void put_real(typename Traits<MODE>::lds_t* dst, long ps, double x) {
  if constexpr (MODE == M_F64) {
    dst[0] = x;
  } else if constexpr (MODE == M_F32) {
    dst[0] = (float)x;
  } else {
    uint16_t h[Traits<MODE>::NPIECE];
    split_d<Traits<MODE>::NPIECE>(x, h);
#pragma unroll
    for (int p = 0; p < Traits<MODE>::NPIECE; ++p) dst[p * ps] = h[p];
  }
}
// Re, Im and -Im into their planes (-Im: the pieces of Im with the sign flipped, exact).
template <int MODE>
__device__ __forceinline__ void put_cplx3(typename Traits<MODE>::lds_t* dst, long ps, double re, double im) {
  constexpr int NP = Traits<MODE>::NPIECE;
  if constexpr (MODE == M_F64) {
    dst[0] = re; dst[ps] = im; dst[2 * ps] = -im;
  } else if constexpr (MODE == M_F32) {
    dst[0] = (float)re; dst[ps] = (float)im; dst[2 * ps] = -(float)im;
  } else {
    uint16_t hr[NP], hi[NP];
    split_d<NP>(re, hr);
    split_d<NP>(im, hi);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      dst[p * ps] = hr[p];
      dst[(NP + p) * ps] = hi[p];
      dst[(2 * NP + p) * ps] = (uint16_t)(hi[p] ^ 0x8000u);
    }
  }
}
template <int MODE>
__device__ __forceinline__ void put_realf(typename Traits<MODE>::lds_t* dst, long ps, float x) {
  if constexpr (MODE == M_F64) {
    dst[0] = (double)x;
  } else if constexpr (MODE == M_F32) {
    dst[0] = x;
  } else {
    uint16_t h[Traits<MODE>::NPIECE];
    split_f<Traits<MODE>::NPIECE>(x, h);
#pragma unroll
    for (int p = 0; p < Traits<MODE>::NPIECE; ++p) dst[p * ps] = h[p];
  }
}

// ---------------------------------------------------------------------------
// MFMA wrappers. A operand: lane l supplies row l%16, k values
// (KS/4)*(l/16) .. +KS/4-1. B operand: lane l supplies column l%16, same k.
// D: lane l, element i holds D[acc_row(l/16, i)][l%16] where the FP32 and BF16
// forms give row 4*(l/16)+i and the FP64 form interleaves, row (l/16)+4*i
// (checked on gfx950 with an in-bounds probe of the builtins).
// ---------------------------------------------------------------------------
template <int MODE>
__device__ __host__ __forceinline__ constexpr int acc_row(int lq, int i) {
  return MODE == M_F64 ? lq + 4 * i : 4 * lq + i;
}
__device__ __forceinline__ d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(u4_t a, u4_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a),
                                                   __builtin_bit_cast(bf8_t, b), c, 0, 0, 0);
}

// x with the sign bits of `mask` flipped (per 32-bit word; bf16 pairs: 0x80008000): a per-lane
// negation without a branch
__device__ __forceinline__ float sign_flip(float x, uint32_t mask) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, x) ^ mask);
}
__device__ __forceinline__ u4_t sign_flip(u4_t x, uint32_t mask) { return x ^ mask; }
__device__ __forceinline__ double negate(double x) { return -x; }
__device__ __forceinline__ float negate(float x) { return -x; }
__device__ __forceinline__ u4_t negate(u4_t x) { return x ^ 0x80008000u; }

// Buffer loads: one scalar resource per item (base, size in bytes), a per-lane
// 32-bit offset and a wave-uniform scalar offset, so that the many loads of a
// K panel share one address register. Offsets at or beyond the size read zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <class OP>
__device__ __forceinline__ OP buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(OP) == 16) {
    return __builtin_bit_cast(OP, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
  } else if constexpr (sizeof(OP) == 8) {
    return __builtin_bit_cast(OP, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  } else {
    return __builtin_bit_cast(OP, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  }
}

// 16 bytes per lane from a buffer straight into LDS: lane l writes lds + 16 l
// (the LDS address must be wave-uniform). A device function, not a lambda: the
// host pass of the compiler has no such builtin.
__device__ __forceinline__ void lds_load16(__amdgpu_buffer_rsrc_t r, void* lds, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, (int)voff,
                                           (int)soff, 0, 0);
}

// Values the whole workgroup shares, moved to scalar registers: loads of them
// are vector loads (the kernel also writes global memory), and buffer
// resources built from vector registers would need a loop over lanes.
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uni(T* p) { return (T*)uni((int64_t)p); }

}  // namespace exc
