// Device twin of the synthetic M generator of synth/__init__.py (inputs only: no
// arithmetic of the exchange method).
//
// One (k, q) block of M is [n''][n][I] (I fastest). Element e = (n'' n_b + n) N_MB + I
// is (z0 + i z1) * exp(-0.1 I / N_MB), where (z0, z1) is the Box-Muller pair built
// from outputs 2e and 2e+1 of the counter-mode SplitMix64 stream (Steele, Lea & Flood,
// OOPSLA 2014) started at the block's seed:
//   output j  = mix64(seed + (j + 1) * 0x9E3779B97F4A7C15)
//   u         = ((output >> 11) + 0.5) / 2^53                 (open interval (0, 1))
//   z0, z1    = r cos t, r sin t,  r = sqrt(-2 ln u_2e),  t = 2 pi u_2e+1
// The host generator evaluates the same expressions in the same order in float64, so
// the two agree to the last bit or two of the double (the device log, sin, cos and exp
// are not the host's); complex64 output rounds each part to nearest even.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double open_unit(uint64_t x) {
  return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

template <bool C64>
__global__ __launch_bounds__(256) void fill_m_kernel(void* dst, uint64_t seed, int64_t n, int32_t nmb) {
  const uint64_t gamma = 0x9E3779B97F4A7C15ull;
  const double two_pi = 6.283185307179586;   // float64 nearest to 2 pi, as math.pi * 2.0
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const uint64_t j = 2ull * (uint64_t)e;
    const double u1 = open_unit(mix64(seed + (j + 1ull) * gamma));
    const double u2 = open_unit(mix64(seed + (j + 2ull) * gamma));
    const double r = sqrt(-2.0 * log(u1));
    const double t = two_pi * u2;
    const double z0 = r * cos(t), z1 = r * sin(t);
    const int64_t I = e % nmb;
    const double d = exp((-0.1 * (double)I) / (double)nmb);
    if (C64) {
      ((float2*)dst)[e] = make_float2((float)(z0 * d), (float)(z1 * d));
    } else {
      ((double2*)dst)[e] = make_double2(z0 * d, z1 * d);
    }
  }
}

}  // namespace

extern "C" {

// Fill one (k, q) block of M: n = n_occ * n_b * N_MB complex elements at dst (device
// memory, complex128 when c64 = 0, complex64 when c64 = 1), from the block's stream seed
// (synth.stream_seed). Asynchronous on `stream` (hipStream_t; NULL = default stream).
// Returns 0, -1 for bad arguments, or -4 if the launch failed.
int synth_fill_m(void* dst, int32_t c64, uint64_t seed, int64_t n, int32_t nmb, void* stream) {
  if (!dst || n < 0 || nmb < 1 || (c64 != 0 && c64 != 1)) return -1;
  if (n == 0) return 0;
  const int64_t blocks = (n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 16384 ? blocks : 16384);
  hipStream_t st = (hipStream_t)stream;
  if (c64)
    hipLaunchKernelGGL(fill_m_kernel<true>, dim3(grid), dim3(256), 0, st, dst, seed, n, nmb);
  else
    hipLaunchKernelGGL(fill_m_kernel<false>, dim3(grid), dim3(256), 0, st, dst, seed, n, nmb);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"
