// One-wavefront measurement of how the gfx950 matrix instructions used by the reduced-precision
// kernels round their accumulation: D = C + sum_k A[0][k] B[k][0] with B = 1, a crafted row 0 of A
// and C[0][0]; prints D[0][0]. Its output is the fixture mfma_rounding_gfx950.json beside this file
// (built and run by hand: hipcc --offload-arch=gfx950 -O2 -o probe mfma_rounding_probe.hip && ./probe).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <vector>

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));

__global__ void probe_bf16(const unsigned short* arow /*32*/, float c00, float* out) {
  const int l = threadIdx.x;
  const int row = l & 15, kq = l >> 4;
  unsigned short a[8], b[8];
  for (int i = 0; i < 8; ++i) {
    a[i] = row == 0 ? arow[8 * kq + i] : 0;
    b[i] = 0x3F80;   // 1.0
  }
  u4_t av, bv;
  memcpy(&av, a, 16);
  memcpy(&bv, b, 16);
  f4_t c = {0, 0, 0, 0};
  if (l == 0) c[0] = c00;
  f4_t d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, av), __builtin_bit_cast(bf8_t, bv), c, 0, 0, 0);
  if (l == 0) out[0] = d[0];
}

__global__ void probe_f32(const float* arow /*4*/, float c00, float* out) {
  const int l = threadIdx.x;
  const int row = l & 15, k = l >> 4;
  const float a = row == 0 ? arow[k] : 0.f;
  f4_t c = {0, 0, 0, 0};
  if (l == 0) c[0] = c00;
  f4_t d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, 1.0f, c, 0, 0, 0);
  if (l == 0) out[0] = d[0];
}

static unsigned short bf(float x) {  // exact bf16 (inputs chosen representable)
  unsigned u;
  memcpy(&u, &x, 4);
  if (u & 0xFFFF) printf("  (not bf16-exact: %a)\n", x);
  return (unsigned short)(u >> 16);
}

int main() {
  unsigned short* da;
  float* dfa;
  float* dout;
  hipMalloc(&da, 64);
  hipMalloc(&dfa, 16);
  hipMalloc(&dout, 4);
  auto run16 = [&](const char* name, std::vector<float> a, float c, const char* expect) {
    unsigned short h[32] = {0};
    for (size_t i = 0; i < a.size() && i < 32; ++i) h[i] = bf(a[i]);
    hipMemcpy(da, h, 64, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(probe_bf16, dim3(1), dim3(64), 0, 0, da, c, dout);
    float r;
    hipMemcpy(&r, dout, 4, hipMemcpyDeviceToHost);
    printf("bf16 %-34s D = %.9g (%a)   [%s]\n", name, r, r, expect);
  };
  auto run4 = [&](const char* name, std::vector<float> a, float c, const char* expect) {
    float h[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < a.size() && i < 4; ++i) h[i] = a[i];
    hipMemcpy(dfa, h, 16, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(probe_f32, dim3(1), dim3(64), 0, 0, dfa, c, dout);
    float r;
    hipMemcpy(&r, dout, 4, hipMemcpyDeviceToHost);
    printf("f32  %-34s D = %.9g (%a)   [%s]\n", name, r, r, expect);
  };
  const float u = ldexpf(1.f, -23);   // ulp of 1
  std::vector<float> z(32, 0.f);
  { auto a = z; a[0] = ldexpf(1.f, -24); run16("C=1 + half ulp", a, 1.f, "RNE 1, RTZ 1, up 1+u"); }
  { auto a = z; a[0] = 3 * ldexpf(1.f, -25); run16("C=1 + 0.75 ulp", a, 1.f, "RNE 1+u, RTZ 1"); }
  { auto a = z; a[0] = ldexpf(1.f, -24) * (1 + ldexpf(1.f, -6)); run16("C=1 + (half+eps) ulp", a, 1.f, "RNE 1+u, RTZ 1"); }
  { auto a = z; a[0] = -3 * ldexpf(1.f, -25); run16("C=1 - 0.75 ulp(1)/1", a, 1.f, "RNE 1-u/2.., RTZ lower"); }
  { auto a = z; for (int k = 0; k < 32; ++k) a[k] = ldexpf(1.f, -28); run16("C=1 + 32 x 2^-28", a, 1.f, "presum 1+u, seq 1"); }
  { auto a = z; for (int k = 0; k < 8; ++k) a[k] = ldexpf(1.f, -26); run16("C=1 + 8 x 2^-26 (k 0-7)", a, 1.f, "presum 1+u"); }
  { auto a = z; for (int k = 0; k < 4; ++k) a[8 * k] = ldexpf(1.f, -25); run16("C=1 + 4 x 2^-25 (one per lane grp)", a, 1.f, "presum 1+u"); }
  { auto a = z; a[0] = 1.f; a[1] = ldexpf(1.f, -30); a[2] = -1.f; run16("C=0: 1 + 2^-30 - 1", a, 0.f, "exact 2^-30"); }
  { auto a = z; a[0] = 1.f; a[9] = ldexpf(1.f, -30); a[17] = -1.f; run16("C=0: 1, 2^-30, -1 (diff lane grps)", a, 0.f, "exact 2^-30"); }
  { auto a = z; a[0] = 1.f; a[1] = -1.f; run16("C=2^24: +1 -1", a, ldexpf(1.f, 24), "presum 2^24, seq 2^24-1"); }
  { auto a = z; a[0] = 1.f; a[1] = ldexpf(1.f, -24); run16("C=0: 1 + 2^-24 (tie)", a, 0.f, "RNE 1"); }
  { auto a = z; a[0] = 1.f; a[1] = 3 * ldexpf(1.f, -25); run16("C=0: 1 + 0.75u", a, 0.f, "RNE 1+u, RTZ 1"); }
  { auto a = z; a[0] = 1.f; a[1] = -3 * ldexpf(1.f, -26); run16("C=0: 1 - 0.75u/2", a, 0.f, "RNE 1-u/2, RTZ 1-u/2?"); }
  { auto a = z; a[0] = 1.f; for (int k = 1; k < 32; ++k) a[k] = ldexpf(1.f, -25); run16("C=0: 1 + 31 x 2^-25", a, 0.f, "exact 1+15.5u"); }
  { auto a = z; a[0] = 1.f; for (int k = 1; k < 32; ++k) a[k] = -ldexpf(1.f, -26); run16("C=0: 1 - 31 x 2^-26", a, 0.f, "exact"); }
  { auto a = z; a[0] = 1.f; for (int k = 1; k < 32; ++k) a[k] = ldexpf(1.f, -26) * 3; run16("C=0: 1 + 31 x 3*2^-26", a, 0.f, "exact"); }
  // FP32 16x16x4
  run4("C=1 + half ulp", {ldexpf(1.f, -24), 0, 0, 0}, 1.f, "RNE 1");
  run4("C=1 + 0.75 ulp", {3 * ldexpf(1.f, -25), 0, 0, 0}, 1.f, "RNE 1+u, RTZ 1");
  run4("C=1 - 0.75 ulp", {-3 * ldexpf(1.f, -25), 0, 0, 0}, 1.f, "");
  run4("C=1 + 4 x 2^-25", {ldexpf(1.f, -25), ldexpf(1.f, -25), ldexpf(1.f, -25), ldexpf(1.f, -25)}, 1.f, "presum 1+u, seq 1");
  run4("C=0: 1 + 2^-30 - 1", {1.f, ldexpf(1.f, -30), -1.f, 0}, 0.f, "exact 2^-30");
  run4("C=2^24: +1 -1", {1.f, -1.f, 0, 0}, ldexpf(1.f, 24), "presum 2^24, seq 2^24-1");
  run4("C=0: 1 + 3*2^-25 + 3*2^-25", {1.f, 3 * ldexpf(1.f, -25), 3 * ldexpf(1.f, -25), 0}, 0.f, "exact 1+1.5u");
  run4("C=0: 1.5*2^-25*... ", {ldexpf(1.f, 0) + ldexpf(1.f, -23), ldexpf(1.f, -24), 0, 0}, 0.f, "1+u + u/2 -> RNE 1+2u");
  (void)u;
  hipFree(da);
  hipFree(dfa);
  hipFree(dout);
  return 0;
}
