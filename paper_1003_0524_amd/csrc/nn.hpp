// Kernels of the learned V^x extrapolator (extension of the nested
// self-consistency scheme of Sec. IV, where V^x is held fixed between outer
// steps): a two-hidden-layer tanh MLP trained with Adam on (dP -> dV) pairs,
// the encoding of dP and dV, and a batched Hermitian eigensolver for the basis
// of the encoding and for judging predictions by their eigenvalues.
//
//   MLP:     h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3,
//            parameters flat as [W1, b1, W2, b2, W3, b3], row-major, FP32;
//            loss = mean squared error over samples and outputs; Adam with
//            beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias correction.
//   GEMMs:   FP32 on MFMA (v_mfma_f32_16x16x4f32), 64x64 block tiles staged
//            through LDS, fused bias / tanh / tanh-derivative epilogues.
//   Encoding: x = Rademacher sketch of vec(P_new - P_old) / |.|; y =
//            enc(B^H (V_a - V_b) B) * scale with B the n_blk eigenvectors of
//            the anchor V for its most negative eigenvalues.
//   Eigen:   cyclic Jacobi with the round-robin parallel ordering, FP64,
//            one workgroup per matrix.
#pragma once
#include "common.hpp"

namespace exc {

// ---------------------------------------------------------------------------
// FP32 GEMM on MFMA: C[M x N] = op(A)[M x K] op(B)[K x N] (+ epilogue).
//   op(A)[i][k] = TA ? A[k*lda + i] : A[i*lda + k]
//   op(B)[k][j] = TB ? B[j*ldb + k] : B[k*ldb + j]
// Epilogues: NONE, BIAS (+bias[j]), BIAS_TANH (tanh(. + bias[j])),
// DTANH (. * (1 - aux[i*ldaux + j]^2)).
// ---------------------------------------------------------------------------
enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3 };

struct GemmArgs {
  const float* A; const float* B; float* C;
  const float* bias; const float* aux;
  int32_t lda, ldb, ldc, ldaux, M, N, K;
};

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void nn_gemm(GemmArgs g) {
  constexpr int BT = 64, KC = 16, LD = BT + 4;
  __shared__ float sA[KC][LD];       // k-major: sA[k][row]
  __shared__ float sB[KC][LD];       // sB[k][col]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;
  const int wr = w & 1, wc = w >> 1;
  const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
  f4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += KC) {
#pragma unroll
    for (int j = 0; j < (BT * KC) / 256; ++j) {
      const int e = tid + 256 * j;
      int r, kk;
      if (TA) { r = e % BT; kk = e / BT; } else { kk = e % KC; r = e / KC; }
      const int gi = m0 + r, gk = k0 + kk;
      float v = 0.f;
      if (gi < g.M && gk < g.K) v = TA ? g.A[(long)gk * g.lda + gi] : g.A[(long)gi * g.lda + gk];
      sA[kk][r] = v;
      int c, kb;
      if (TB) { kb = e % KC; c = e / KC; } else { c = e % BT; kb = e / BT; }
      const int gj = n0 + c, gkb = k0 + kb;
      float u = 0.f;
      if (gj < g.N && gkb < g.K) u = TB ? g.B[(long)gj * g.ldb + gkb] : g.B[(long)gkb * g.ldb + gj];
      sB[kb][c] = u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sA[kk + lq][wr * 32 + i * 16 + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sB[kk + lq][wc * 32 + j * 16 + l16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wr * 32 + i * 16 + acc_row<M_F32>(lq, e);
        const int col = n0 + wc * 32 + j * 16 + l16;
        if (row < g.M && col < g.N) {
          float v = acc[i][j][e];
          if (EPI == EPI_BIAS) v += g.bias[col];
          if (EPI == EPI_BIAS_TANH) v = tanhf(v + g.bias[col]);
          if (EPI == EPI_DTANH) {
            const float h = g.aux[(long)row * g.ldaux + col];
            v *= 1.f - h * h;
          }
          g.C[(long)row * g.ldc + col] = v;
        }
      }
}

// g[j] = sum_i D[i*ld + j], i < n (bias gradients), fixed order.
__global__ __launch_bounds__(256) void nn_colsum(const float* D, int ld, int n, int ncol, float* g) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= ncol) return;
  float s = 0.f;
  for (int i = 0; i < n; ++i) s += D[(long)i * ld + j];
  g[j] = s;
}

// dY = 2 (Y - T) / (n O); loss = mean (Y - T)^2; also advances the Adam step
// counter (read by nn_adam, which runs after this kernel on the same stream).
__global__ __launch_bounds__(256) void nn_loss_grad(const float* Y, const float* T, float* dY, long cnt,
                                                     float* loss, int32_t* step, int advance) {
  __shared__ double red[256];
  double s = 0.0;
  const float sc = 2.f / (float)cnt;
  for (long e = threadIdx.x; e < cnt; e += 256) {
    const float d = Y[e] - T[e];
    dY[e] = sc * d;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *loss = (float)(red[0] / (double)cnt);
    if (advance) *step += 1;
  }
}

__global__ __launch_bounds__(256) void nn_adam(float* theta, const float* grad, float* m, float* v, long n,
                                                const int32_t* step, float lr) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int t = *step;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float bc1 = (float)(1.0 - pow(0.9, (double)t));
  const float bc2 = (float)(1.0 - pow(0.999, (double)t));
  const float gi = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// SplitMix64 (Steele, Lea & Flood 2014), output i of the counter stream.
__device__ __host__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Initial parameters: weights (2u - 1)/sqrt(fan_in), u = top 53 bits / 2^53 of
// the stream output at the flat index; biases zero.
struct InitArgs { long off[7]; int fan[3]; };
__global__ __launch_bounds__(256) void nn_init_params(float* theta, InitArgs a, uint64_t seed) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.off[6]) return;
  int seg = 0;
  while (seg < 5 && i >= a.off[seg + 1]) ++seg;
  if (seg & 1) { theta[i] = 0.f; return; }
  const double u = (double)(splitmix64_at(seed, (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
  theta[i] = (float)((2.0 * u - 1.0) / sqrt((double)a.fan[seg >> 1]));
}

// ---------------------------------------------------------------------------
// Sketch of dP = P_new - P_old: s_i = sum_j S_ij v_j with S_ij = -1 when the
// top bit of SplitMix64(seed) output i*D + j is set, else +1; v_j runs over
// (k', column, row, re/im) of the n_kp complex n_b x n_b matrices. Pass 1: one
// partial vector per chunk of v; pass 2: fixed-order sum, scaling by
// 1/(sqrt(m) |v|).
// ---------------------------------------------------------------------------
constexpr int SK_CHUNK = 2048;
constexpr int SK_MMAX = 128;

__global__ __launch_bounds__(256) void nn_sketch_partial(const double* Pn, const double* Po, long D,
                                                          int m, uint64_t seed, double* part) {
  __shared__ double v[SK_CHUNK];
  __shared__ double red[256];
  const long j0 = (long)blockIdx.x * SK_CHUNK;
  const int len = (int)min((long)SK_CHUNK, D - j0);
  double sq = 0.0;
  for (int j = threadIdx.x; j < SK_CHUNK; j += 256) {
    double x = 0.0;
    if (j < len) x = Pn[j0 + j] - Po[j0 + j];
    v[j] = x;
    sq += x * x;
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  double* out = part + (long)blockIdx.x * (m + 1);
  if (threadIdx.x == 0) out[m] = red[0];
  // each output row i: 256/m threads (at least one) split the chunk; fixed order
  const int per = max(1, 256 / m);
  for (int base = 0; base < m; base += 256 / per) {
    const int i = base + threadIdx.x / per, sub = threadIdx.x % per;
    double s = 0.0;
    if (i < m) {
      const uint64_t row0 = (uint64_t)i * (uint64_t)D + (uint64_t)j0;
      for (int j = sub; j < len; j += per) {
        const uint64_t r = splitmix64_at(seed, row0 + (uint64_t)j);
        s += (r >> 63) ? -v[j] : v[j];
      }
    }
    __syncthreads();
    red[threadIdx.x] = s;
    __syncthreads();
    if (i < m && sub == 0) {
      double t = 0.0;
      for (int q = 0; q < per; ++q) t += red[threadIdx.x + q];
      out[i] = t;
    }
  }
}

__global__ __launch_bounds__(128) void nn_sketch_final(const double* part, int nchunk, int m, float* x,
                                                        double* norm_out) {
  __shared__ double nrm;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nchunk; ++b) s += part[(long)b * (m + 1) + m];
    nrm = sqrt(s);
    *norm_out = nrm;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += 128) {
    double s = 0.0;
    for (int b = 0; b < nchunk; ++b) s += part[(long)b * (m + 1) + i];
    x[i] = nrm > 0.0 ? (float)(s / (sqrt((double)m) * nrm)) : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Projection y_k = enc(B_k^H (Va_k - Vb_k) B_k) * scale and expansion
// V_out = V_anchor + scale * B_k dec(y_k) B_k^H. B_k = first n_blk columns of
// the n x n column-major eigenvector matrix Z_k. enc: R[i][j] = Re H_ij (i <= j),
// R[j][i] = Im H_ij (i < j), row-major n_blk x n_blk.
// ---------------------------------------------------------------------------
struct ProjArgs {
  const double2* const* Va; const double2* const* Vb;  // [n_k] device pointers
  const double2* Z; const int64_t* z_off;             // packed eigenvectors, offsets per k
  const int32_t* nb;                                  // n_b per k
  int32_t n_blk; double scale;
  float* y;                                           // [n_k][n_blk^2]
  const double2* const* Vanc; double2* const* Vout;   // expansion
};

__device__ __forceinline__ double2 cfma_conj_a(double2 a, double2 b, double2 acc) {   // acc + conj(a) b
  return make_double2(acc.x + a.x * b.x + a.y * b.y, acc.y + a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 acc) {          // acc + a b
  return make_double2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(256) void nn_project(ProjArgs a) {
  extern __shared__ double2 W[];                      // [n_blk][n]: (Va - Vb) B, column-major
  const int k = blockIdx.x, n = a.nb[k], nbk = a.n_blk;
  const double2* B = a.Z + a.z_off[k];
  const double2* Va = a.Va[k];
  const double2* Vb = a.Vb[k];
  for (int e = threadIdx.x; e < n * nbk; e += 256) {
    const int r = e % n, c = e / n;
    double2 s = make_double2(0.0, 0.0);
    for (int t = 0; t < n; ++t) {
      const double2 va = Va[r + (long)t * n], vb = Vb[r + (long)t * n];
      s = cfma(make_double2(va.x - vb.x, va.y - vb.y), B[t + (long)c * n], s);
    }
    W[r + c * n] = s;
  }
  __syncthreads();
  float* y = a.y + (long)k * nbk * nbk;
  for (int e = threadIdx.x; e < nbk * nbk; e += 256) {
    const int i = e / nbk, j = e % nbk;
    if (i > j) continue;
    double2 h = make_double2(0.0, 0.0);
    for (int t = 0; t < n; ++t) h = cfma_conj_a(B[t + (long)i * n], W[t + j * n], h);
    y[i * nbk + j] = (float)(h.x * a.scale);
    if (i < j) y[j * nbk + i] = (float)(h.y * a.scale);
  }
}

__global__ __launch_bounds__(256) void nn_expand(ProjArgs a) {
  extern __shared__ double2 T[];                      // [n][n_blk]: T = H B^H, stored T[c*nbk + i]
  const int k = blockIdx.x, n = a.nb[k], nbk = a.n_blk;
  const double2* B = a.Z + a.z_off[k];
  const float* y = a.y + (long)k * nbk * nbk;
  for (int e = threadIdx.x; e < n * nbk; e += 256) {
    const int i = e % nbk, c = e / nbk;
    double2 s = make_double2(0.0, 0.0);
    for (int j = 0; j < nbk; ++j) {
      double2 h;
      if (i == j) h = make_double2((double)y[i * nbk + i], 0.0);
      else if (i < j) h = make_double2((double)y[i * nbk + j], (double)y[j * nbk + i]);
      else h = make_double2((double)y[j * nbk + i], -(double)y[i * nbk + j]);
      const double2 b = B[c + (long)j * n];
      s = cfma(h, make_double2(b.x, -b.y), s);       // H_ij conj(B_cj)
    }
    T[c * nbk + i] = s;
  }
  __syncthreads();
  const double2* V0 = a.Vanc[k];
  double2* Vo = a.Vout[k];
  for (long e = threadIdx.x; e < (long)n * n; e += 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < nbk; ++i) s = cfma(B[r + (long)i * n], T[c * nbk + i], s);
    const double2 v0 = V0[e];
    Vo[e] = make_double2(v0.x + a.scale * s.x, v0.y + a.scale * s.y);
  }
}

// ---------------------------------------------------------------------------
// Batched Hermitian eigensolver: cyclic Jacobi, round-robin parallel ordering.
// Each round applies n/2 disjoint plane rotations at once: A <- A G then
// A <- G^H A, Z <- Z G. For the pair (p, q), with b = A_pq = |b| e^{i phi},
// D = diag(1, e^{-i phi}) makes the 2x2 block real symmetric and the classic
// symmetric Schur rotation (tau = (A_qq - A_pp)/(2|b|), t = sign(tau)/(|tau| +
// sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c) diagonalises it:
// G = D [[c, s], [-s, c]]. Stops when the off-diagonal Frobenius norm falls
// below 1e-14 of the full norm, or after 50 sweeps. Output: ascending
// eigenvalues and the matching columns of Z.
// ---------------------------------------------------------------------------
struct EighArgs {
  const double2* const* A;     // [n_mat] input matrices (column-major, Hermitian)
  const int32_t* n;            // [n_mat] orders
  double2* work;               // packed working copies (offsets z_off)
  double2* Z;                  // packed eigenvectors (offsets z_off)
  const int64_t* z_off;
  double* w;                   // packed eigenvalues (offsets w_off)
  const int64_t* w_off;
  int32_t* sweeps;             // [n_mat] sweeps used
};

constexpr int EIGH_NMAX = 256;

__global__ __launch_bounds__(256) void eigh_jacobi(EighArgs a) {
  __shared__ double rc[EIGH_NMAX / 2], rs[EIGH_NMAX / 2];
  __shared__ double2 rph[EIGH_NMAX / 2];
  __shared__ int rp[EIGH_NMAX / 2], rq[EIGH_NMAX / 2];
  __shared__ double red[256];
  __shared__ int done;
  __shared__ int order[EIGH_NMAX];
  const int mtx = blockIdx.x, n = a.n[mtx], tid = threadIdx.x;
  double2* A = a.work + a.z_off[mtx];
  double2* Z = a.Z + a.z_off[mtx];
  const double2* A0 = a.A[mtx];
  for (long e = tid; e < (long)n * n; e += 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    // Hermitian part of the input
    const double2 x = A0[e], y = A0[c + (long)r * n];
    A[e] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    Z[e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int ne = n + (n & 1);              // even number of players, the extra one sits out
  const int npair = ne / 2;
  int sweep = 0;
  for (; sweep < 50; ++sweep) {
    // convergence test on the current matrix
    double off = 0.0, tot = 0.0;
    for (long e = tid; e < (long)n * n; e += 256) {
      const int r = (int)(e % n), c = (int)(e / n);
      const double m2 = A[e].x * A[e].x + A[e].y * A[e].y;
      tot += m2;
      if (r != c) off += m2;
    }
    red[tid] = off;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0) done = (offs <= 1e-28 * red[0]) || n < 2;
    __syncthreads();
    if (done) break;
    for (int round = 0; round < ne - 1; ++round) {
      // circle method: player ne-1 fixed, the others rotate
      for (int i = tid; i < npair; i += 256) {
        int p, q;
        if (i == 0) { p = ne - 1; q = round; }
        else { p = (round + i) % (ne - 1); q = (round - i + (ne - 1)) % (ne - 1); }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        double2 ph = make_double2(1.0, 0.0);      // e^{-i phi}
        if (q < n) {
          const double2 b = A[p + (long)q * n];
          const double ab = sqrt(b.x * b.x + b.y * b.y);
          if (ab > 0.0) {
            ph = make_double2(b.x / ab, -b.y / ab);
            const double app = A[p + (long)p * n].x, aqq = A[q + (long)q * n].x;
            const double tau = (aqq - app) / (2.0 * ab);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        rp[i] = p; rq[i] = q; rc[i] = c; rs[i] = s; rph[i] = ph;
      }
      __syncthreads();
      // columns: A <- A G, Z <- Z G with G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
      for (long e = tid; e < (long)npair * n; e += 256) {
        const int r = (int)(e % n), i = (int)(e / n);
        const int p = rp[i], q = rq[i];
        if (q >= n || rs[i] == 0.0) continue;
        const double c = rc[i], s = rs[i];
        const double2 ph = rph[i];
        for (int mat = 0; mat < 2; ++mat) {
          double2* X = mat ? Z : A;
          const double2 xp = X[r + (long)p * n], xq = X[r + (long)q * n];
          const double2 xqph = make_double2(xq.x * ph.x - xq.y * ph.y, xq.x * ph.y + xq.y * ph.x);
          X[r + (long)p * n] = make_double2(c * xp.x - s * xqph.x, c * xp.y - s * xqph.y);
          X[r + (long)q * n] = make_double2(s * xp.x + c * xqph.x, s * xp.y + c * xqph.y);
        }
      }
      __syncthreads();
      // rows: A <- G^H A: row p = c A_p - s e^{i phi} A_q, row q = s A_p + c e^{i phi} A_q
      for (long e = tid; e < (long)npair * n; e += 256) {
        const int col = (int)(e % n), i = (int)(e / n);
        const int p = rp[i], q = rq[i];
        if (q >= n || rs[i] == 0.0) continue;
        const double c = rc[i], s = rs[i];
        const double2 phc = make_double2(rph[i].x, -rph[i].y);   // e^{i phi}
        const double2 ap = A[p + (long)col * n], aq = A[q + (long)col * n];
        const double2 aqph = make_double2(aq.x * phc.x - aq.y * phc.y, aq.x * phc.y + aq.y * phc.x);
        A[p + (long)col * n] = make_double2(c * ap.x - s * aqph.x, c * ap.y - s * aqph.y);
        A[q + (long)col * n] = make_double2(s * ap.x + c * aqph.x, s * ap.y + c * aqph.y);
      }
      __syncthreads();
      // the rotated pairs are now diagonal blocks: clean the rounding residue
      for (int i = tid; i < npair; i += 256) {
        const int p = rp[i], q = rq[i];
        if (q >= n || rs[i] == 0.0) continue;
        A[p + (long)q * n] = make_double2(0.0, 0.0);
        A[q + (long)p * n] = make_double2(0.0, 0.0);
        A[p + (long)p * n].y = 0.0;
        A[q + (long)q * n].y = 0.0;
      }
      __syncthreads();
    }
  }
  // ascending order (stable selection by one thread; n <= EIGH_NMAX)
  if (tid == 0) {
    for (int i = 0; i < n; ++i) order[i] = i;
    for (int i = 1; i < n; ++i) {
      const int o = order[i];
      const double v = A[o + (long)o * n].x;
      int j = i - 1;
      while (j >= 0 && A[order[j] + (long)order[j] * n].x > v) { order[j + 1] = order[j]; --j; }
      order[j + 1] = o;
    }
    a.sweeps[mtx] = sweep;
  }
  __syncthreads();
  double* w = a.w + a.w_off[mtx];
  for (int i = tid; i < n; i += 256) w[i] = A[order[i] + (long)order[i] * n].x;
  __syncthreads();
  // permute the columns of Z through the (now free) working copy
  for (long e = tid; e < (long)n * n; e += 256) A[e] = Z[e];
  __syncthreads();
  for (long e = tid; e < (long)n * n; e += 256) {
    const int r = (int)(e % n), c = (int)(e / n);
    Z[e] = A[r + (long)order[c] * n];
  }
}

}  // namespace exc
