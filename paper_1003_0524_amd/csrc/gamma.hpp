// Gamma-point term of the exchange matrix (Sec. III.E, eqs. "F(q)", "divergence",
// "div final"). The 1/q^2 part of the Coulomb matrix, damped by exp(-beta q^2),
// is integrated analytically; what the q-mesh sum already holds is subtracted:
//
//   C = erf(sqrt(beta) q0) / sqrt(pi beta)
//       - 4 pi / (N Omega) * sum_{p, 0 < |p| <= q0} exp(-beta |p|^2) / |p|^2,
//
// p over every point q + G of the q mesh, i.e. every p = j0 g0 + j1 g1 + j2 g2
// with integer j and g_i = b_i / mesh_i; exp(-beta q0^2) = beta. V_nn gains
// -C for the occupied bands (occupation 1 per spin).
//
// The sum is ALU work (one exp and one reciprocal in FP64 per point, nothing
// read from memory): a wavefront takes one line (j0, j1) at a time, its lanes
// the consecutive j2 of the part of the line that meets the sphere (found from
// the quadratic in j2, widened by one point on each side; the membership test
// itself is exact per point). Lines go to wavefronts round-robin over a fixed
// grid and partial sums are reduced in a fixed order, so the result does not
// depend on timing.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace exc {

struct GammaArgs {
  double g[3][3];        // rows g_i = b_i / mesh_i (bohr^-1)
  double beta, q0sq;
  int32_t J[3];          // box half-widths: |j_i| <= J_i holds every point with |p| <= q0
  double* part;          // [2 * gridDim.x]: per-workgroup sum and term count
};

constexpr int kGammaBlock = 256;
constexpr int kGammaGrid = 2048;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kGammaBlock) void gamma_sum_kernel(GammaArgs a) {
  __shared__ double red[2][kGammaBlock / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t n1 = 2 * (int64_t)a.J[1] + 1;
  const int64_t n_lines = (2 * (int64_t)a.J[0] + 1) * n1;
  const int64_t waves = (int64_t)gridDim.x * (kGammaBlock / 64);
  const double g2x = a.g[2][0], g2y = a.g[2][1], g2z = a.g[2][2];
  const double gg = g2x * g2x + g2y * g2y + g2z * g2z, inv_gg = 1.0 / gg;
  const double dead = -1e-9 * gg * a.q0sq;
  // (i0, i1) of the line, advanced by the grid's stride without a division per line
  int64_t line = (int64_t)blockIdx.x * (kGammaBlock / 64) + wv;
  int64_t i0 = line / n1, i1 = line % n1;
  const int64_t s0 = waves / n1, s1 = waves % n1;
  double acc = 0.0, cnt = 0.0;
  for (; line < n_lines; line += waves) {
    const double j0 = (double)(i0 - a.J[0]);
    const double j1 = (double)(i1 - a.J[1]);
    i0 += s0;
    i1 += s1;
    if (i1 >= n1) {
      i1 -= n1;
      ++i0;
    }
    const double px = j0 * a.g[0][0] + j1 * a.g[1][0];
    const double py = j0 * a.g[0][1] + j1 * a.g[1][1];
    const double pz = j0 * a.g[0][2] + j1 * a.g[1][2];
    // |p0 + t g2|^2 <= q0^2  <=>  gg t^2 + 2 b t + c <= 0
    const double b = px * g2x + py * g2y + pz * g2z;
    const double c = px * px + py * py + pz * pz - a.q0sq;
    const double disc = b * b - gg * c;
    if (disc < dead) continue;                                   // wavefront-uniform
    const double half = sqrt(fmax(disc, 0.0)) * inv_gg, tc = -b * inv_gg;
    const int lo = max(-a.J[2], (int)floor(tc - half) - 1);
    const int hi = min(a.J[2], (int)ceil(tc + half) + 1);
    for (int t = lo + lane; t <= hi; t += 64) {
      const double j2 = (double)t;
      const double x = px + j2 * g2x, y = py + j2 * g2y, z = pz + j2 * g2z;
      const double p2 = x * x + y * y + z * z;
      if (p2 > 0.0 && p2 <= a.q0sq) {
        // 1/p2: hardware estimate and two Newton steps (within an ulp of the quotient;
        // p2 lies in [|g|_min^2, q0^2], far from denormals and overflow)
        double rp = __builtin_amdgcn_rcp(p2);
        rp = fma(rp, fma(-p2, rp, 1.0), rp);
        rp = fma(rp, fma(-p2, rp, 1.0), rp);
        acc = fma(exp(-a.beta * p2), rp, acc);
        cnt += 1.0;
      }
    }
  }
  acc = wave_sum(acc);
  cnt = wave_sum(cnt);
  if (lane == 0) {
    red[0][wv] = acc;
    red[1][wv] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, n = 0.0;
    for (int w = 0; w < kGammaBlock / 64; ++w) {
      s += red[0][w];
      n += red[1][w];
    }
    a.part[2 * blockIdx.x] = s;
    a.part[2 * blockIdx.x + 1] = n;
  }
}

// One workgroup: the partials in a fixed order, then C.
//   out[0] = C, out[1] = lattice sum, out[2] = number of terms, out[3] = diagonal
//   shift the q-sum applies (C if apply, else 0).
__global__ __launch_bounds__(kGammaBlock) void gamma_finish_kernel(const double* part, int n_part, double beta,
                                                                   double q0, double pref, int apply,
                                                                   double* out) {
  __shared__ double red[2][kGammaBlock];
  double s = 0.0, n = 0.0;
  for (int i = threadIdx.x; i < n_part; i += kGammaBlock) {
    s += part[2 * i];
    n += part[2 * i + 1];
  }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = n;
  __syncthreads();
  for (int h = kGammaBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pi = 3.14159265358979323846;
    const double C = erf(sqrt(beta) * q0) / sqrt(pi * beta) - pref * red[0][0];
    out[0] = C;
    out[1] = red[0][0];
    out[2] = red[1][0];
    out[3] = apply ? C : 0.0;
  }
}

}  // namespace exc
