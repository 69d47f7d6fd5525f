// Auxiliary kernels: block-sparse rows, FP64 reduction, energy, Cholesky of
// v(q) and preparation of the dense factor in the product mode's storage.
#pragma once
#include "common.hpp"
#include "tile.hpp"

namespace exc {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {   // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// ---------------------------------------------------------------------------
// Block-sparse rows of the transformed mixed product basis (Fig. 1): each
// multipole-free MT function couples only to the functions of its own
// (atom, L, M) channel, i.e. to the other multipole-free functions of the
// channel and to the channel's multipole function.
//   HERK form: Y_c = L_c^H A_c + l_c a_{j(c)}   (rows of L^H A for v = L L^H)
//   GEMM form: W_c = D_c A_c + C_c a_{j(c)},  X_c = C_c^H A_c (added to W row j(c))
// The MT and multipole rows of a column (k, q, n'', n) are staged in LDS with
// coalesced loads, every row is computed in FP64 and written once, so the kernel
// is bound by HBM bandwidth. GEMM form: one wavefront per column, four per
// workgroup. HERK form: a workgroup is one wavefront that takes NCW columns of a
// pair at once (their loads all in flight together, no barrier), and the row
// r = first + i of channel c reads its coefficient run L_c[i..b-1][i] once for
// the NCW columns, eight values per round of loads, from a copy of the runs
// stored entry by entry (the lanes of a round, consecutive rows, read
// consecutive addresses). Output: double2
// rows (FP64 mode), or (reduced-precision modes) the whole column packed into
// the tile kernel's split planes [plane][row]: the sparse rows Y_s followed by
// the dense rows of M, each part zero padded (this is also the conversion of M
// to the product mode's storage, done once per column).
// ---------------------------------------------------------------------------
struct SparseArgs {
  const PairInfo* pairs;
  const void* const* mtab;
  int32_t m_c64;
  int32_t n_s, n_ch, n_occ, nb_max;
  int32_t ns_pad;            // n_s rounded up to 8: start of the dense rows in a packed column
  const int32_t* row_chan;   // [n_s] channel of each multipole-free row
  const int32_t* ch_off;     // [n_ch] first multipole-free row of the channel
  const int32_t* ch_len;     // [n_ch] nrad - 1
  const int64_t* ch_coef;    // [n_ch] offset of the channel's square block in coef
  const double2* coef;       // HERK: L_c (lower, col-major); GEMM: D_c (col-major)
  const double2* cvec;       // [n_s] HERK: l_c = L_c^{-1} C_c; GEMM: C_c
  const int4* rowinfo;       // [n_s] HERK: {start of the row's run in coef, run length b - i,
                             //  multipole row n_s + c, 0}
  const double2* runs;       // HERK: [run_max][runs_ld] entry t of row r's run conj-coefficients
  int32_t run_max, runs_ld;  //  L_c[i + t][i] at runs[t * runs_ld + r] (zero past the run)
  int64_t runs_qs;           //  elements between the copies of q and q + 1 (0: one copy)
  int64_t coef_qs, cvec_qs;  // elements between the copies of q and q + 1 (0: one copy for all q)
  void* ws;                  // output rows
  double* dsp;               // HERK, reduced precision: sum_r |Y_s[r][n]|^2 per column
};

// The column's nrow multipole-free and multipole rows to S: eight loads per lane
// issued before the first LDS write (the last row stands in for rows past the end).
__device__ __forceinline__ void stage_column(double2* S, const char* mb, long mcol, int nrow, int m_c64,
                                             int lane) {
  for (int r0 = 0; r0 < nrow; r0 += 8 * 64) {
    double2 v[8];
    if (m_c64) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float2 f = ((const float2*)mb)[mcol + min(r0 + u * 64 + lane, nrow - 1)];
        v[u] = make_double2(f.x, f.y);
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = ((const double2*)mb)[mcol + min(r0 + u * 64 + lane, nrow - 1)];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r0 + u * 64 + lane < nrow) S[r0 + u * 64 + lane] = v[u];
  }
}

// HERK form: NCW columns (k, q, n'', n), n'' n consecutive, of one pair per single-wavefront
// workgroup. The columns' rows go to LDS (complex128 M: straight from HBM, every load of
// every column in flight at once; complex64 M: through registers), then each round of
// 64 rows reads its coefficient runs once for all NCW columns.
template <int MODE, int NCW>
__device__ __forceinline__ void herk_columns(const SparseArgs& a, double2* scol) {
  const int lane = threadIdx.x;
  const PairInfo pi = a.pairs[blockIdx.y];
  const int ncol = a.n_occ * pi.nb, c0 = (int)blockIdx.x * NCW;
  if (c0 >= ncol) return;
  const int nc = min(NCW, ncol - c0);                  // columns of this workgroup (the rest idle)
  const int n_s = a.n_s, nrow = n_s + a.n_ch, nrp = (nrow + 63) & ~63;
  const double2* cvec = a.cvec + pi.q * a.cvec_qs;
  const double2* runs = a.runs + pi.q * a.runs_qs;
  if (nrow > 0) {
    const char* mb = (const char*)a.mtab[pi.k];
    if (a.m_c64) {
      for (int j = 0; j < nc; ++j)
        stage_column(scol + j * nrp, mb, pi.m_off + (long)(c0 + j) * pi.nmb, nrow, 1, lane);
    } else {
      // rows past nrow read zero (offsets beyond the resource's size)
      for (int j = 0; j < nc; ++j) {
        const auto rs = make_rsrc(uni(mb + (pi.m_off + (long)(c0 + j) * pi.nmb) * 16), (uint32_t)nrow * 16);
        for (int u = 0; u < nrp / 64; ++u) lds_load16(rs, scol + j * nrp + u * 64, (uint32_t)lane * 16, u * 1024);
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);    // vmcnt(0): the columns have landed in LDS
    }
  }
  // LDS operations of one wavefront take effect in order: the rows just written are
  // read below by other lanes of the same wavefront
  __builtin_amdgcn_wave_barrier();
  const int nr = MODE == M_F64 ? n_s : a.ns_pad;       // FP64: Y_s; else the packed sparse part
  double dsum[NCW];
#pragma unroll
  for (int j = 0; j < NCW; ++j) dsum[j] = 0.0;
  int4 ri = make_int4(0, 1, 0, 0);
  double2 cv = make_double2(0.0, 0.0);
  if (lane < n_s) { ri = a.rowinfo[lane]; cv = cvec[lane]; }
  for (int r = lane; r < nr; r += 64) {
    // next round's row descriptors first
    int4 rn = make_int4(0, 1, 0, 0);
    double2 cn = make_double2(0.0, 0.0);
    if (r + 64 < n_s) { rn = a.rowinfo[r + 64]; cn = cvec[r + 64]; }
    // Y_s[r] = sum_{t < len} conj(L_c[i + t][i]) A[r + t] + l_c[i] A[multipole row of c]:
    // eight loads of the run per round, unconditional (indices clamped into the table and
    // the run), the terms past the run add zero
    double2 y[NCW];
#pragma unroll
    for (int j = 0; j < NCW; ++j) y[j] = make_double2(0.0, 0.0);
    if (r < n_s) {
      const double2* run = runs + r;
      for (int t0 = 0; t0 < ri.y; t0 += 8) {
        double2 cf[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) cf[u] = run[(long)min(t0 + u, a.run_max - 1) * a.runs_ld];
        int sr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const bool in = t0 + u < ri.y;
          cf[u] = make_double2(in ? cf[u].x : 0.0, in ? cf[u].y : 0.0);
          sr[u] = r + min(t0 + u, ri.y - 1);
        }
#pragma unroll
        for (int j = 0; j < NCW; ++j) {
          double2 sv[8];                     // the column's eight rows, all requested at once
#pragma unroll
          for (int u = 0; u < 8; ++u) sv[u] = scol[j * nrp + sr[u]];
#pragma unroll
          for (int u = 0; u < 8; ++u) y[j] = cadd(y[j], cmulc(cf[u], sv[u]));
        }
      }
#pragma unroll
      for (int j = 0; j < NCW; ++j) y[j] = cadd(y[j], cmul(cv, scol[j * nrp + ri.z]));
    }
#pragma unroll
    for (int j = 0; j < NCW; ++j) {
      if (j >= nc) break;
      const int col = c0 + j;
      if constexpr (MODE == M_F64) {
        ((double2*)a.ws)[pi.ws_off + (long)col * pi.ldw + r] = y[j];
      } else {
        using lds_t = typename Traits<MODE>::lds_t;
        constexpr int NP = Traits<MODE>::NPIECE;
        lds_t* out = (lds_t*)a.ws + pi.ws_off + (long)col * 2 * NP * pi.ldw;
        dsum[j] += y[j].x * y[j].x + y[j].y * y[j].y;
        put_real<MODE>(out + r, pi.ldw, y[j].x);
        put_real<MODE>(out + (long)NP * pi.ldw + r, pi.ldw, y[j].y);
      }
    }
    ri = rn;
    cv = cn;
  }
  if constexpr (MODE != M_F64) {
    // the dense rows A_d of M into the packed column (zero beyond N_d), and the FP64
    // sums of |Y_s|^2 per column
    using lds_t = typename Traits<MODE>::lds_t;
    constexpr int NP = Traits<MODE>::NPIECE;
    const char* mb = (const char*)a.mtab[pi.k];
#pragma unroll
    for (int j = 0; j < NCW; ++j) {
      if (j >= nc) break;
      const int col = c0 + j;
      lds_t* out = (lds_t*)a.ws + pi.ws_off + (long)col * 2 * NP * pi.ldw;
      const long mcol = pi.m_off + (long)col * pi.nmb + n_s;
      for (int d = lane; d < pi.ldw - a.ns_pad; d += 64) {
        double2 x = make_double2(0.0, 0.0);
        if (d < pi.nd) {
          if (a.m_c64) {
            const float2 v = ((const float2*)mb)[mcol + d];
            x = make_double2(v.x, v.y);
          } else {
            x = ((const double2*)mb)[mcol + d];
          }
        }
        put_real<MODE>(out + a.ns_pad + d, pi.ldw, x.x);
        put_real<MODE>(out + (long)NP * pi.ldw + a.ns_pad + d, pi.ldw, x.y);
      }
      double ds = dsum[j];
      for (int o = 32; o > 0; o >>= 1) ds += __shfl_xor(ds, o);
      if (lane == 0) a.dsp[(long)blockIdx.y * a.n_occ * a.nb_max + col] = ds;
    }
  }
}

// HERK form: herk_columns (one wavefront per workgroup). GEMM form (FP64 only): four
// wavefronts, one column each.
template <int FORM, int MODE, int NCW = 1>
__global__ __launch_bounds__(256) void sparse_kernel(SparseArgs a) {
  extern __shared__ double2 scol[];          // HERK: [NCW][nrow rounded up to 64]; GEMM: [4 waves][nrow]
  if constexpr (FORM == 1) {
    herk_columns<MODE, NCW>(a, scol);
  } else {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const PairInfo pi = a.pairs[blockIdx.y];
    const double2* coef = a.coef + pi.q * a.coef_qs;      // this q's channel blocks
    const double2* cvec = a.cvec + pi.q * a.cvec_qs;
    const int col = (int)blockIdx.x * 4 + w;
    const bool active = col < a.n_occ * pi.nb;
    const int nrow = a.n_s + a.n_ch;
    double2* S = scol + (long)w * nrow;
    if (active && nrow > 0)
      stage_column(S, (const char*)a.mtab[pi.k], pi.m_off + (long)col * pi.nmb, nrow, a.m_c64, lane);
    __syncthreads();
    if (!active) return;                     // whole wavefronts leave; no barrier follows
    const long wcol = pi.ws_off + (long)col * pi.ldw;
    double2* out = (double2*)a.ws;
    for (int r = lane; r < a.n_s; r += 64) {
      const int c = a.row_chan[r], s = a.ch_off[c], b = a.ch_len[c], i = r - s;
      const double2* cf = coef + a.ch_coef[c];
      double2 y = make_double2(0.0, 0.0);
      for (int j = 0; j < b; ++j) y = cadd(y, cmul(cf[i + (long)j * b], S[s + j]));
      out[wcol + r] = cadd(y, cmul(cvec[r], S[a.n_s + c]));
    }
    for (int c = lane; c < a.n_ch; c += 64) {
      const int s = a.ch_off[c], b = a.ch_len[c];
      double2 x = make_double2(0.0, 0.0);
      for (int j = 0; j < b; ++j) x = cadd(x, cmulc(cvec[s + j], S[s + j]));
      out[wcol + a.n_s + c] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 reduction of the item partials of each k:
//   V(k) = - sum_{slots of k} w_q(slot) * (Gram tiles of the slot)
// with the Hermitian mirror and Im V_nn = 0. One workgroup per (Gram tile, k):
// 64 entries of the 8x8 band block times 4 interleaved slot subsets, combined
// in a fixed order. In the reduced-precision HERK modes the diagonal comes from
// the FP64 sums of |Y|^2.
// ---------------------------------------------------------------------------
struct ReduceArgs {
  const int32_t* k_nb;         // [n_k]
  const int32_t* slot_begin;   // [n_k + 1]
  const double* slot_w;        // [n_slots]
  const void* gpart;
  int32_t gstride, acc64;
  const double* dpart;
  int32_t dstride, use_d64;
  double2* vres;
  const int64_t* v_off;        // [n_k]
  void* const* vout;           // [n_k] device pointers or nullptr
  const double* gshift;        // Gamma-point term added to -V_nn for n < n_occ (0 when unset)
  int32_t n_occ;
  int32_t real_v;              // 1: V = Re of the result (inversion symmetry, packed real bands)
  int32_t* counter;            // work counters of the persistent launch before this one, cleared
  int32_t n_counter;           // here for the next launch (nullptr / 0: none)
};

// Slot groups per q-sum workgroup: group sg sums slots sg, sg + RED_SG, ... of its k
// (one round of loads for up to 6 RED_SG slots), the groups are added in order.
constexpr int RED_SG = 16;

// Position of G[row][col] of Gram tile tp in a partial slot written as
// [tile][element i][lane] (see acc_row for the two accumulator layouts).
template <int ACC64>
__device__ __forceinline__ int gidx(int tp, int row, int col) {
  return ACC64 ? (tp * 4 + (row >> 2)) * 64 + col + 16 * (row & 3)
               : (tp * 4 + (row & 3)) * 64 + col + 16 * (row >> 2);
}

template <int ACC64>
__global__ __launch_bounds__(64 * RED_SG) void reduce_kernel(ReduceArgs a) {
  __shared__ double red[RED_SG][64][3];
  if (blockIdx.x == 0 && blockIdx.y == 0 && (int)threadIdx.x < a.n_counter) a.counter[threadIdx.x] = 0;
  const int k = blockIdx.y;
  const int nb = a.k_nb[k];
  const int nbt = (nb + 7) >> 3;
  const int tp = blockIdx.x;
  if (tp >= nbt * (nbt + 1) / 2) return;     // uniform over the workgroup
  int I, J;
  tp_to_ij(tp, I, J);
  const int e = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int c = e & 7, c2 = e >> 3;
  const int n = I * 8 + c, n2 = J * 8 + c2;
  const int irr = gidx<ACC64>(tp, c, c2), iii = gidx<ACC64>(tp, c + 8, c2 + 8);
  const int iri = gidx<ACC64>(tp, c, c2 + 8), iir = gidx<ACC64>(tp, c + 8, c2);
  double re = 0.0, im = 0.0, dg = 0.0;
  // slots sg, sg + RED_SG, ... in order; UN slots' loads are issued before their adds,
  // unconditionally: a slot past the end reads the last slot of k and weighs it by zero
  constexpr int UN = 6;
  const int s0 = a.slot_begin[k] + sg, s1 = a.slot_begin[k + 1];
  const bool use_d = a.use_d64 != 0;
  const int nc = min(n, nb - 1);             // (the diagonal entry of this lane's column)
  for (int sb = s0; sb < s1; sb += RED_SG * UN) {
    double wq[UN], grr[UN], gii[UN], gri[UN], gir[UN], dd[UN];
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      const int s = sb + RED_SG * u, sc = min(s, s1 - 1);
      const double w = a.slot_w[sc];
      wq[u] = s < s1 ? w : 0.0;
      if (ACC64) {
        const double* g = (const double*)a.gpart + (long)sc * a.gstride;
        grr[u] = g[irr]; gii[u] = g[iii]; gri[u] = g[iri]; gir[u] = g[iir];
      } else {
        const float* g = (const float*)a.gpart + (long)sc * a.gstride;
        grr[u] = g[irr]; gii[u] = g[iii]; gri[u] = g[iri]; gir[u] = g[iir];
      }
      dd[u] = use_d ? a.dpart[(long)sc * a.dstride + nc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UN; ++u) {
      re += wq[u] * (grr[u] + gii[u]);
      im += wq[u] * (gri[u] - gir[u]);
      dg += wq[u] * dd[u];
    }
  }
  red[sg][e][0] = re;
  red[sg][e][1] = im;
  red[sg][e][2] = dg;
  __syncthreads();
  if (sg != 0 || n >= nb || n2 >= nb || n > n2) return;
  re = red[0][e][0];
  im = red[0][e][1];
  double dsum = red[0][e][2];
#pragma unroll
  for (int g = 1; g < RED_SG; ++g) {
    re += red[g][e][0];
    im += red[g][e][1];
    dsum += red[g][e][2];
  }
  if (a.real_v) im = 0.0;
  if (n == n2) {
    im = 0.0;
    if (a.use_d64) re = dsum;
    if (n < a.n_occ) re += *a.gshift;
  }
  const double2 v = make_double2(-re, -im);
  double2* V = a.vres + a.v_off[k];
  V[n + (long)n2 * nb] = v;
  if (n != n2) V[n2 + (long)n * nb] = make_double2(-re, im);
  if (a.vout && a.vout[k]) {
    double2* O = (double2*)a.vout[k];
    O[n + (long)n2 * nb] = v;
    if (n != n2) O[n2 + (long)n * nb] = make_double2(-re, im);
  }
}

// ---------------------------------------------------------------------------
// Energy: per k, Tr(rho_k V_k) (or 2 sum_{n < n_occ} V_nn for rho = 2 P_occ),
// reduced in a fixed order; the host applies 1/2 sum_k w_k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void energy_kernel(const double2* vres, const int64_t* v_off,
                                                     const int32_t* k_nb, const void* const* rho,
                                                     int32_t n_occ, double* out) {
  __shared__ double red[256];
  const int k = blockIdx.x, nb = k_nb[k];
  const double2* V = vres + v_off[k];
  double s = 0.0;
  const double2* R = rho ? (const double2*)rho[k] : nullptr;
  if (R) {
    for (long e = threadIdx.x; e < (long)nb * nb; e += 256) {
      const int n = (int)(e % nb), n2 = (int)(e / nb);
      const double2 r = R[e];                      // rho[n][n2]
      const double2 v = V[n2 + (long)n * nb];      // V[n2][n]
      s += r.x * v.x - r.y * v.y;
    }
  } else {
    for (int n = threadIdx.x; n < n_occ && n < nb; n += 256) s += 2.0 * V[n + (long)n * nb].x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = red[0];
}

// E_x for rho_k = diag(2 for n < n_occ): 1/2 sum_k w_k sum_{n < n_occ} 2 Re V_k[n][n], in one
// workgroup: thread t takes the (k, n) pairs t, t + 256, ... and the partial sums are
// combined by a fixed tree.
__global__ __launch_bounds__(256) void energy_diag_kernel(const double2* vres, const int64_t* v_off,
                                                          const int32_t* k_nb, int32_t n_k, int32_t n_occ,
                                                          const double* w_k, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n_k * n_occ; i += 256) {
    const int k = i / n_occ, n = i - k * n_occ, nb = k_nb[k];
    if (n < nb) s += (w_k ? w_k[k] : 1.0 / n_k) * 2.0 * vres[v_off[k] + n + (long)n * nb].x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5 * red[0];
}

// E_x = 1/2 sum_k w_k e_k on the device, in the fixed order of k (one workgroup).
__global__ __launch_bounds__(256) void energy_sum_kernel(const double* e_k, const double* w_k, int32_t n_k,
                                                         double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n_k; k += 256) s += (w_k ? w_k[k] : 1.0 / n_k) * e_k[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5 * red[0];
}

// ---------------------------------------------------------------------------
// Per-channel factorisation (HERK form, q independent): D_c = L_c L_c^H,
// l_c = L_c^{-1} C_c and the Schur update ||l_c||^2 of the channel's multipole
// diagonal entry. With one multipole function per channel the Schur
// complement E - C^H D^{-1} C changes only those diagonal entries.
// ---------------------------------------------------------------------------
// blockIdx.y: the copy of the channel blocks (one per q when they depend on q), strides in
// elements between copies.
__global__ void chan_chol_kernel(int n_ch, const int32_t* ch_off, const int32_t* ch_len,
                                 const int64_t* ch_coef, double2* L, double2* lvec,
                                 double* schur, int* info, int64_t coef_qs, int64_t cvec_qs) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_ch) return;
  L += blockIdx.y * coef_qs;
  lvec += blockIdx.y * cvec_qs;
  schur += (long)blockIdx.y * n_ch;
  const int b = ch_len[c], s = ch_off[c];
  double2* A = L + ch_coef[c];
  for (int j = 0; j < b; ++j) {
    double d = A[j + (long)j * b].x;
    for (int p = 0; p < j; ++p) {
      const double2 x = A[j + (long)p * b];
      d -= x.x * x.x + x.y * x.y;
    }
    if (!(d > 0.0)) { atomicMax(info, 1); d = 1.0; }
    d = sqrt(d);
    A[j + (long)j * b] = make_double2(d, 0.0);
    for (int i = j + 1; i < b; ++i) {
      double2 t = A[i + (long)j * b];
      for (int p = 0; p < j; ++p) {
        const double2 u = cmul(A[i + (long)p * b], make_double2(A[j + (long)p * b].x, -A[j + (long)p * b].y));
        t.x -= u.x; t.y -= u.y;
      }
      A[i + (long)j * b] = make_double2(t.x / d, t.y / d);
    }
    for (int i = 0; i < j; ++i) A[i + (long)j * b] = make_double2(0.0, 0.0);
  }
  double sc = 0.0;
  for (int i = 0; i < b; ++i) {
    double2 t = lvec[s + i];
    for (int p = 0; p < i; ++p) {
      const double2 u = cmul(A[i + (long)p * b], lvec[s + p]);
      t.x -= u.x; t.y -= u.y;
    }
    const double d = A[i + (long)i * b].x;
    t = make_double2(t.x / d, t.y / d);
    lvec[s + i] = t;
    sc += t.x * t.x + t.y * t.y;
  }
  schur[c] = sc;
}

// ---------------------------------------------------------------------------
// Dense Cholesky of the (Schur-updated) block E(q) = L22 L22^H, FP64, one
// workgroup per q, left-looking with 16-column panels.
// ---------------------------------------------------------------------------
struct CholArgs {
  double2* A;             // per-q matrices (column-major, leading dimension lda)
  const int64_t* a_off;
  const int32_t* nd;
  const int32_t* lda;
  int32_t n_ch;
  const double* schur;    // [n_ch] (per q: [n_q][n_ch]) or nullptr
  int32_t schur_qs;       // n_ch when the channel blocks depend on q, else 0
  int* info;              // [n_q] first failing pivot (1-based), 0 = ok
};

// threads per q of the dense Cholesky (one row of the panel update per thread: more rows in
// flight hide the latency of their loads)
constexpr int kCholThreads = 512;
__global__ __launch_bounds__(kCholThreads) void dense_chol_kernel(CholArgs a) {
  constexpr int NTC = kCholThreads;
  constexpr int NB = 16, PC = 32;
  static_assert(PC % 8 == 0, "panel stage: whole groups of eight values");
  __shared__ double2 Lp[NB][PC + 1];
  __shared__ double2 Ld[NB][NB + 1];
  __shared__ int s_fail;
  const int q = blockIdx.x, tid = threadIdx.x;
  const int n = a.nd[q], lda = a.lda[q];
  double2* A = a.A + a.a_off[q];
  if (tid == 0) s_fail = 0;
  if (a.schur)
    for (int c = tid; c < a.n_ch && c < n; c += NTC) A[c + (long)c * lda].x -= a.schur[(long)q * a.schur_qs + c];
  __syncthreads();
  for (int jb = 0; jb < n; jb += NB) {
    const int nbk = min(NB, n - jb);
    // panel update: A[i][jb+jj] -= sum_{p<jb} A[i][p] conj(A[jb+jj][p]),  i >= jb
    for (int i0 = jb; i0 < n; i0 += NTC) {
      const int i = i0 + tid;
      double2 acc[NB];
#pragma unroll
      for (int jj = 0; jj < NB; ++jj) acc[jj] = make_double2(0.0, 0.0);
      for (int p0 = 0; p0 < jb; p0 += PC) {
        __syncthreads();
        for (int e = tid; e < NB * PC; e += NTC) {
          const int jj = e / PC, pp = e % PC;
          Lp[jj][pp] = (jj < nbk && p0 + pp < jb) ? A[(jb + jj) + (long)(p0 + pp) * lda] : make_double2(0.0, 0.0);
        }
        __syncthreads();
        if (i < n) {
          // eight values of the row requested together (past the panel's end: zeros, against the
          // zero-filled stage), then their products
          const int pe = min(PC, jb - p0);
          for (int pp0 = 0; pp0 < pe; pp0 += 8) {
            double2 xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              xv[u] = pp0 + u < pe ? A[i + (long)(p0 + pp0 + u) * lda] : make_double2(0.0, 0.0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const double2 x = xv[u];
#pragma unroll
              for (int jj = 0; jj < NB; ++jj) {
                const double2 y = Lp[jj][pp0 + u];
                acc[jj].x += x.x * y.x + x.y * y.y;
                acc[jj].y += x.y * y.x - x.x * y.y;
              }
            }
          }
        }
      }
      if (i < n) {
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {           // (fixed bound: acc stays in registers)
          if (jj < nbk) {
            double2* t = &A[i + (long)(jb + jj) * lda];
            t->x -= acc[jj].x; t->y -= acc[jj].y;
          }
        }
      }
    }
    __syncthreads();
    // factor the diagonal block in LDS
    for (int e = tid; e < NB * NB; e += NTC) {
      const int r = e % NB, cc = e / NB;
      Ld[r][cc] = (r < nbk && cc < nbk) ? A[(jb + r) + (long)(jb + cc) * lda] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (tid == 0) {
      for (int j = 0; j < nbk; ++j) {
        double d = Ld[j][j].x;
        for (int p = 0; p < j; ++p) d -= Ld[j][p].x * Ld[j][p].x + Ld[j][p].y * Ld[j][p].y;
        if (!(d > 0.0)) { if (!s_fail) s_fail = jb + j + 1; d = 1.0; }
        d = sqrt(d);
        Ld[j][j] = make_double2(d, 0.0);
        for (int i = j + 1; i < nbk; ++i) {
          double2 t = Ld[i][j];
          for (int p = 0; p < j; ++p) {
            t.x -= Ld[i][p].x * Ld[j][p].x + Ld[i][p].y * Ld[j][p].y;
            t.y -= Ld[i][p].y * Ld[j][p].x - Ld[i][p].x * Ld[j][p].y;
          }
          Ld[i][j] = make_double2(t.x / d, t.y / d);
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < nbk * nbk; e += NTC) {
      const int r = e % nbk, cc = e / nbk;
      if (r >= cc) A[(jb + r) + (long)(jb + cc) * lda] = Ld[r][cc];
    }
    // rows below: x Ld^H = a  ->  x_j = (a_j - sum_{m<j} x_m conj(Ld[j][m])) / Ld[j][j]
    for (int i = jb + nbk + tid; i < n; i += NTC) {
      // an index offset of zero the compiler cannot see through: the block's values are read
      // from LDS per row instead of being hoisted into (spilled) registers for all rows
      int zb = 0;
      asm volatile("" : "+v"(zb));
      const double2* Lz = &Ld[0][0] + zb;
      double2 x[NB];
      for (int j = 0; j < NB; ++j) x[j] = j < nbk ? A[i + (long)(jb + j) * lda] : make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        if (j < nbk) {
          double2 t = x[j];
#pragma unroll
          for (int m = 0; m < NB; ++m) {
            if (m < j) {
              const double2 l = Lz[j * (NB + 1) + m];
              t.x -= x[m].x * l.x + x[m].y * l.y;
              t.y -= x[m].y * l.x - x[m].x * l.y;
            }
          }
          const double d = Lz[j * (NB + 1) + j].x;
          x[j] = make_double2(t.x / d, t.y / d);
          A[i + (long)(jb + j) * lda] = x[j];       // (stored here: x stays in registers)
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) a.info[q] = s_fail;
}

// ---------------------------------------------------------------------------
// Write the dense factor of q into the tile kernel's planes:
//   HERK: B[r][c] = conj(L22[c][r]) for c >= r (upper triangular L22^H)
//   GEMM: B[r][c] = E[r][c]
// planes [re pieces..., im pieces...], each ldu x ldu row-major, zero padded.
// ---------------------------------------------------------------------------
template <int MODE, int FORM>
__global__ __launch_bounds__(256) void prep_factor_kernel(const double2* src, const int64_t* s_off,
                                                          const int32_t* nd, const int32_t* lds,
                                                          void* dst, const int64_t* d_off,
                                                          const int32_t* ldu) {
  using lds_t = typename Traits<MODE>::lds_t;
  constexpr int NP = Traits<MODE>::NPIECE;
  const int q = blockIdx.y;
  const int n = nd[q], ld = ldu[q], ls = lds[q];
  const long plane = (long)ld * ld;
  lds_t* D = (lds_t*)dst + d_off[q];
  const double2* S = src + s_off[q];
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < plane; e += (long)gridDim.x * 256) {
    const int r = (int)(e / ld), c = (int)(e % ld);
    double re = 0.0, im = 0.0;
    if (r < n && c < n) {
      if (FORM == 1) {
        if (c >= r) {
          const double2 v = S[c + (long)r * ls];
          re = v.x; im = -v.y;
        }
      } else {
        const double2 v = S[r + (long)c * ls];
        re = v.x; im = v.y;
      }
    }
    put_real<MODE>(D + e, plane, re);
    put_real<MODE>(D + NP * plane + e, plane, im);
  }
}

// Padded copy of each multipole-free row's coefficient run, transposed per
// chunk of 32 rows: out[((r / 32) * mt + t) * 32 + r % 32] = coef[rowinfo[r].x + t]
// for t < min(rowinfo[r].y, mt), zero beyond (and for the padding rows of the
// last chunk). Lanes that hold consecutive rows then read consecutive entries.
__global__ __launch_bounds__(256) void pad_runs_kernel(const double2* coef, const int4* rowinfo,
                                                       const int4* chunks, int nchunk, int mt, int gr,
                                                       double2* out, int64_t coef_qs) {
  // blockIdx.y: the copy of the channel blocks (its padded runs follow the previous copy's)
  coef += blockIdx.y * coef_qs;
  out += (long)blockIdx.y * nchunk * mt * gr;
  // out[chunk][t][rr] = L_c[i+t][i] of the chunk's row rr (entry i of channel c), zero past the run
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)nchunk * mt * gr) return;
  const int rr = (int)(e % gr), t = (int)((e / gr) % mt), ck = (int)(e / ((long)gr * mt));
  const int4 ci = chunks[ck];
  double2 v = make_double2(0.0, 0.0);
  if (rr < ci.y) {
    const int4 ri = rowinfo[ci.x + rr];
    if (t < ri.y) v = coef[ri.x + t];
  }
  out[e] = v;
}

// sparse_kernel's copy of the factored channel coefficients: out[t][r] (row stride ld) =
// L_c[i+t][i] for the multipole-free row r (entry i of channel c) and t < b - i, zero beyond
// and for the padding rows r >= n_s. blockIdx.y: the copy of the channel blocks.
__global__ __launch_bounds__(256) void runs_by_row_kernel(const double2* coef, const int4* rowinfo, int n_s,
                                                          int rmax, int ld, double2* out, int64_t coef_qs) {
  coef += blockIdx.y * coef_qs;
  out += (long)blockIdx.y * rmax * ld;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)rmax * ld) return;
  const int r = (int)(e % ld), t = (int)(e / ld);
  double2 v = make_double2(0.0, 0.0);
  if (r < n_s) {
    const int4 ri = rowinfo[r];
    if (t < ri.y) v = coef[ri.x + t];
  }
  out[e] = v;
}

}  // namespace exc
