// Back-transform of V^x(k) to the LAPW basis (Sec. III.A, eq. "APW trafo"):
//   V_GG = Z V Z^H,  Z = S c  (n_G x n_b, S the overlap matrix, c the eigenvectors).
//
// Two launches. bt_left_kernel forms T = Z V (n_G x n_b, small: FP64 VALU, one
// thread per element). bt_gram_kernel forms the n_G x n_G product T Z^H on FP64
// MFMA in 64 x 64 tiles: wavefront w of a workgroup owns 16 columns of its tile
// and the tile's 64 rows as four 16 x 16 blocks, each complex block built from
// four real 16x16x4 products; operands come straight from T and Z (L2-resident,
// n_b <= 128), 16 values of n per round of loads, and the tile is written once
// with the 16 lanes of a row group storing 16 consecutive rows of a column (256
// contiguous bytes). Output bytes
// dominate for n_b < ~20 (the product has n_b / 2 flop per output byte against
// the FP64 ridge of ~10), the MFMA work beyond.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.hpp"

namespace exc {

// T[g + n * nG] = sum_m Z[g + m * nG] V[m + n * nb]
__global__ __launch_bounds__(256) void bt_left_kernel(const double2* __restrict__ Z, const double2* __restrict__ V,
                                                      int nG, int nb, double2* __restrict__ T) {
  const int g = blockIdx.x * 256 + threadIdx.x, n = blockIdx.y;
  if (g >= nG) return;
  double re = 0.0, im = 0.0;
#pragma unroll 8
  for (int m = 0; m < nb; ++m) {                  // (eight loads of Z in flight)
    const double2 z = Z[g + (long)m * nG], v = V[m + (long)n * nb];
    re = fma(z.x, v.x, re);
    re = fma(-z.y, v.y, re);
    im = fma(z.x, v.y, im);
    im = fma(z.y, v.x, im);
  }
  T[g + (long)n * nG] = make_double2(re, im);
}

// C[b + a * nG] = sum_n T[b + n * nG] conj(Z[a + n * nG]) over 64 x 64 tiles: tile t
// has rows b in (t % nt) * 64 + [0, 64) and columns a in (t / nt) * 64 + [0, 64).
// As an MFMA product D[a][b] = sum_n conj(Z)[a][n] T[b][n]: the A operand is a
// 16 x 4 block of conj(Z) (lane l: column a = l % 16, n = l / 16), the B operand a
// 4 x 16 block of T^T (lane l: row b = l % 16, same n), and lane l holds
// D[l / 16 + 4 i][l % 16] for i < 4, i.e. C[b0 + l % 16][a0 + l / 16 + 4 i].
__global__ __launch_bounds__(256) void bt_gram_kernel(const double2* __restrict__ T, const double2* __restrict__ Z,
                                                      int nG, int nb, double2* __restrict__ C) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int nt = (nG + 63) / 64;
  // tiles in turn (grid-stride): the stores of one tile drain while the next one's
  // operands load and its MFMAs run
  for (int tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
    const int a0 = (tile / nt) * 64 + 16 * w;       // this wavefront's 16 columns of C
    const int bt0 = (tile % nt) * 64;                // the tile's 64 rows of C
    const int a_l = a0 + r16;
    d4_t accr[4], acci[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) accr[j] = acci[j] = d4_t{0.0, 0.0, 0.0, 0.0};
    // K in chunks of 16: the chunk's operands (4 of Z, 16 of T per lane) are requested
    // before its 64 MFMAs, one memory latency per chunk
    for (int n0 = 0; n0 < nb; n0 += 16) {
      const int ns = min(4, (nb - n0 + 3) >> 2);     // MFMA steps of 4 in this chunk (uniform)
      double2 z[4], t[4][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int n = n0 + 4 * s + kq;
        z[s] = (a_l < nG && n < nb) ? Z[a_l + (long)n * nG] : make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int b_l = bt0 + 16 * j + r16;
          t[s][j] = (b_l < nG && n < nb) ? T[b_l + (long)n * nG] : make_double2(0.0, 0.0);
        }
      }
      // conj(z) t = (zr tr + zi ti) + i (zr ti - zi tr)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (s >= ns) break;                            // (no MFMAs on the zero tail of n)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          accr[j] = mfma(z[s].x, t[s][j].x, accr[j]);
          accr[j] = mfma(z[s].y, t[s][j].y, accr[j]);
          acci[j] = mfma(z[s].x, t[s][j].y, acci[j]);
          acci[j] = mfma(-z[s].y, t[s][j].x, acci[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int b = bt0 + 16 * j + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = a0 + kq + 4 * i;
        if (a < nG && b < nG) C[b + (long)a * nG] = make_double2(accr[j][i], acci[j][i]);
      }
    }
  }
}

}  // namespace exc
