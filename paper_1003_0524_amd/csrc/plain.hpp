// FP64 complex products on the matrix cores for the GEMM form of the vector-matrix-
// vector product (Sec. III.C, eq. "vec-mat-vec"), taken one (k, q) pair at a time:
//
//   W   = v(q) A               block-sparse rows (sparse_kernel<0>), dense rows
//                              W_d = E(q) A_d + X on MFMA (zgemm_kernel)
//   G_b = A_b^H W_b            for every occupied n'' = b, on MFMA (zgemm_kernel,
//                              conjugated left operand, split over the MPB index)
//   V  += -w_q sum_b G_b       FP64, fixed order (pair_accumulate_kernel)
//
// and, once the pairs of k are done, V(k) with its Hermitian mirror
// (pair_finish_kernel).
//
// zgemm_kernel computes C = op(A) op(B) for complex operands whose contraction index k
// is contiguous in memory: A(m, k) and B(k, n) each at base + (m or n) * ld + k, in
// complex128 or complex64, optionally conjugated, or A as two row-major FP64 planes
// (real, imaginary) as the prepared Coulomb block E(q) is stored. Complex products on
// the real FP64 16x16x4 MFMA: a 16-column tile holds 8 complex columns, real parts in
// columns 0-7 and imaginary parts in 8-15, and [Cr | Ci] += Ar [Br | Bi] + Ai [-Bi | Br].
// Each workgroup (4 wavefronts in a 2 x 2 grid) owns a BM x BNC tile of C; K panels of
// KC move global -> registers one panel ahead and then to LDS (two buffers, one barrier
// per panel).
#pragma once
#include "common.hpp"

namespace exc {

struct ZgemmArgs {
  // A(m, k): a_kind 0 -> planes: Re = a[m lda + k], Im = a[a_plane + m lda + k] (double);
  //          a_kind 1 -> complex at a + m lda + k (complex64 if a_c64), conjugated if a_conj
  const void* a;
  int64_t lda, a_plane, a_bstride;
  int32_t a_kind, a_c64, a_conj;
  // B(k, n) = complex at b + n ldb + k (complex64 if b_c64), conjugated if b_conj
  const void* b;
  int64_t ldb, b_bstride;
  int32_t b_c64, b_conj;
  // C(m, n) at c + m + n ldc (complex128); batch gridDim.y, K split gridDim.z
  double2* c;
  int64_t ldc, c_bstride, c_sstride;
  int32_t M, N, K;
  int32_t kchunk;            // K range of one split (a multiple of KC)
  int32_t upper;             // 1: only tiles that meet the upper triangle (m <= n)
  int32_t tri_a;             // 1: A(m, k) = 0 for k < m: a tile's K loop starts at its first row
  int32_t add_rows;          // rows m < add_rows: C += result (the multipole rows' C_c^H A_c)
  int32_t a_rows_alloc;      // a_kind 0: rows (and k) readable without bounds checks (zero padded)
};

template <int BM, int BNC, int KC>
struct ZgCfg {
  static constexpr int NT = 256, WR = 2, WC = 2;
  static constexpr int RT = BM / (16 * WR);      // row tiles per wavefront
  static constexpr int CT = BNC / (8 * WC);      // complex column tiles (8 each) per wavefront
  static constexpr int LDK = KC + 2;             // doubles per LDS row (pad: 16 bytes)
  static constexpr int APL = BM * LDK, BPL = BNC * LDK;
  static constexpr int STAGE = 2 * (APL + BPL);  // doubles of one buffer (Re and Im planes)
  static constexpr int AV = BM * KC / NT;        // A elements per thread and panel
  static constexpr int BV = BNC * KC / NT;       // B elements per thread and panel
  static_assert(RT >= 1 && CT >= 1 && BM % 32 == 0 && BNC % 16 == 0, "2 x 2 wavefronts of whole tiles");
  static_assert((BM * KC) % NT == 0 && (BNC * KC) % NT == 0, "whole elements per thread");
  static constexpr size_t LDS_B = (size_t)2 * STAGE * sizeof(double);
};

template <int BM, int BNC, int KC, int OCC>
__global__ __launch_bounds__(256, OCC) void zgemm_kernel(ZgemmArgs g) {
  using Z = ZgCfg<BM, BNC, KC>;
  constexpr int RT = Z::RT, CT = Z::CT, LDK = Z::LDK, APL = Z::APL, BPL = Z::BPL;
  __shared__ __align__(16) double smem[2 * Z::STAGE];

  const int ntn = (g.N + BNC - 1) / BNC;
  const int tm = (int)blockIdx.x / ntn, tn = (int)blockIdx.x % ntn;
  const int m0 = tm * BM, n0 = tn * BNC;
  if (g.upper && m0 > n0 + BNC - 1) return;      // below the diagonal: uniform, before any barrier
  const int bt = blockIdx.y, sp = blockIdx.z;
  int k_lo = sp * g.kchunk;
  const int k_hi = min(g.K, k_lo + g.kchunk);
  if (g.tri_a) k_lo = max(k_lo, m0 / KC * KC);
  const int npan = k_hi > k_lo ? (k_hi - k_lo + KC - 1) / KC : 0;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w % 2, wc = w / 2;
  const int l16 = lane & 15, lq = lane >> 4, c8 = l16 & 7, part = l16 >> 3;

  const char* ab = (const char*)g.a + (g.a_kind == 0 ? (int64_t)bt * g.a_bstride * 8
                                                      : (int64_t)bt * g.a_bstride * (g.a_c64 ? 8 : 16));
  const char* bb = (const char*)g.b + (int64_t)bt * g.b_bstride * (g.b_c64 ? 8 : 16);
  const double asg = g.a_conj ? -1.0 : 1.0, bsg = g.b_conj ? -1.0 : 1.0;

  double2 ra[Z::AV], rb[Z::BV];
  // panel at k0 into registers: element e = tid + NT j of the A panel is (row e / KC, k e % KC)
  auto fetch = [&](int k0) {
#pragma unroll
    for (int j = 0; j < Z::AV; ++j) {
      const int e = tid + Z::NT * j, r = e / KC, kk = e % KC;
      const int m = m0 + r, k = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (g.a_kind == 0) {
        if (m < g.a_rows_alloc && k < g.a_rows_alloc) {
          const double* p = (const double*)ab + (int64_t)m * g.lda + k;
          v = make_double2(p[0], p[g.a_plane]);
        }
      } else if (m < g.M && k < k_hi) {
        if (g.a_c64) {
          const float2 f = ((const float2*)ab)[(int64_t)m * g.lda + k];
          v = make_double2((double)f.x, (double)f.y);
        } else {
          v = ((const double2*)ab)[(int64_t)m * g.lda + k];
        }
      }
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < Z::BV; ++j) {
      const int e = tid + Z::NT * j, cn = e / KC, kk = e % KC;
      const int n = n0 + cn, k = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (n < g.N && k < k_hi) {
        if (g.b_c64) {
          const float2 f = ((const float2*)bb)[(int64_t)n * g.ldb + k];
          v = make_double2((double)f.x, (double)f.y);
        } else {
          v = ((const double2*)bb)[(int64_t)n * g.ldb + k];
        }
      }
      rb[j] = v;
    }
  };
  auto stage = [&](double* S) {
#pragma unroll
    for (int j = 0; j < Z::AV; ++j) {
      const int e = tid + Z::NT * j, r = e / KC, kk = e % KC;
      S[r * LDK + kk] = ra[j].x;
      S[APL + r * LDK + kk] = asg * ra[j].y;
    }
    double* SB = S + 2 * APL;
#pragma unroll
    for (int j = 0; j < Z::BV; ++j) {
      const int e = tid + Z::NT * j, cn = e / KC, kk = e % KC;
      SB[cn * LDK + kk] = rb[j].x;
      SB[BPL + cn * LDK + kk] = bsg * rb[j].y;
    }
  };

  d4_t acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = d4_t{0, 0, 0, 0};

  if (npan > 0) {
    fetch(k_lo);
    stage(smem);
    __syncthreads();
  }
  for (int p = 0; p < npan; ++p) {
    double* S = smem + (p & 1) * Z::STAGE;
    if (p + 1 < npan) fetch(k_lo + (p + 1) * KC);
    const double* SA = S;
    const double* SB = S + 2 * APL;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + lq;
      double ar[RT], ai[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int r = wr * RT * 16 + i * 16 + l16;
        ar[i] = SA[r * LDK + kk];
        ai[i] = SA[APL + r * LDK + kk];
      }
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        const int cn = wc * CT * 8 + j * 8 + c8;
        const double br = SB[cn * LDK + kk], bi = SB[BPL + cn * LDK + kk];
        const double b0 = part ? bi : br;       // [Br | Bi]
        const double b1 = part ? br : -bi;      // [-Bi | Br]
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], b0, acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], b1, acc[i][j], 0, 0, 0);
        }
      }
    }
    if (p + 1 < npan) stage(smem + ((p + 1) & 1) * Z::STAGE);
    __syncthreads();
  }

  double2* cb = g.c + (int64_t)bt * g.c_bstride + (int64_t)sp * g.c_sstride;
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int n = n0 + wc * CT * 8 + j * 8 + c8;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wr * RT * 16 + i * 16 + lq + 4 * e;   // FP64 accumulator row order
        if (m < g.M && n < g.N) {
          double* d = (double*)(cb + m + (int64_t)n * g.ldc) + part;
          const double v = acc[i][j][e];
          *d = m < g.add_rows ? *d + v : v;
        }
      }
    }
}

// V(k) accumulator, upper triangle n <= n': acc = (first ? 0 : acc) - w_q sum_s sum_b G[s][b],
// G[s][b] an nb x nb column-major partial (split s of the MPB index, occupied band b).
__global__ __launch_bounds__(256) void pair_accumulate_kernel(const double2* G, int nsplit, int nocc, int nb,
                                                              double wq, int first, double2* vacc) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nb * nb) return;
  const int n = e % nb, n2 = e / nb;
  if (n > n2) return;
  double re = 0.0, im = 0.0;
  const int64_t nb2 = (int64_t)nb * nb;
  for (int s = 0; s < nsplit; ++s)
    for (int b = 0; b < nocc; ++b) {
      const double2 v = G[((int64_t)s * nocc + b) * nb2 + e];
      re += v.x;
      im += v.y;
    }
  double2 a = first ? make_double2(0.0, 0.0) : vacc[e];
  a.x -= wq * re;
  a.y -= wq * im;
  vacc[e] = a;
}

// V(k) from the accumulated upper triangle: the lower triangle is its conjugate mirror,
// Im V_nn = 0 (and Im V = 0 for real systems), -C on the occupied diagonal when the
// Gamma-point shift is set. Written to the resident V and, if given, the caller's buffer.
// Band-pair tiles the mask of k leaves out (tmask: bit J(J+1)/2 + I of 8 x 8 tile (I, J)) are zero.
__global__ __launch_bounds__(256) void pair_finish_kernel(const double2* vacc, int nb, int n_occ,
                                                          const double* gshift, int real_v, const uint64_t* tmask,
                                                          double2* vres, double2* vout) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nb * nb) return;
  const int n = e % nb, n2 = e / nb;
  if (n > n2) return;
  double2 v = vacc[e];
  const int tp = (n2 >> 3) * ((n2 >> 3) + 1) / 2 + (n >> 3);
  if (tp < 192 && !((tmask[tp >> 6] >> (tp & 63)) & 1)) v = make_double2(0.0, 0.0);
  if (real_v) v.y = 0.0;
  if (n == n2) {
    v.y = 0.0;
    if (n < n_occ) v.x -= *gshift;
  }
  vres[e] = v;
  if (vout) vout[e] = v;
  if (n != n2) {
    const double2 m = make_double2(v.x, -v.y);
    vres[n2 + (int64_t)n * nb] = m;
    if (vout) vout[n2 + (int64_t)n * nb] = m;
  }
}

}  // namespace exc
