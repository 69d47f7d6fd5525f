// Fused dense tile kernel: Y = B A on MFMA for the dense rows of the mixed
// product basis, followed in the same workgroup by the contraction
// G += Left^H Right over the rows of the tile.
//
//   HERK form (v = L L^H):  B = L22^H (upper triangular), Left = Right = Y.
//   GEMM form:              B = E(q) (full), Right = W = E A_d + X, Left = A_d.
//
// The product with v(q) and the band contraction are the two stages of the
// vector-matrix-vector form (Sec. II.C, eq. "vec-mat-vec"); the dense block is
// the "one big block" of multipole functions and plane waves of Fig. 1.
//
// Complex arithmetic on real MFMA: the 16 real columns of one MFMA tile hold
// 8 complex columns, real parts in tile columns 0-7 and imaginary parts in
// 8-15. Y = B A is computed as two real products over the k index,
//   [Yr | Yi] += Br [Ar | Ai] + Bi [-Ai | Ar],
// so a complex multiply-add costs 4 real multiply-adds and odd band counts
// waste at most 7 columns.
//
// Partials: each work item (pair (k,q), a group of n'' values, a range of row
// blocks) accumulates 16x16 real Gram tiles G(I,J), I <= J over 8-column band
// tiles, and writes them (plus, in the reduced-precision modes, an FP64 sum of
// |Y|^2 per band) to its own slot. A separate kernel sums the slots of each k
// in a fixed order in FP64 (deterministic).
#pragma once
#include "common.hpp"

namespace exc {

struct PairInfo {
  int32_t k, q, nb, nmb;   // k, q, bands n_b(k), N_MB(q)
  int32_t nd, nsb, nb8, ndb; // N_d(q), sparse row blocks, n_b rounded to 8, dense row blocks
  int64_t m_off;           // complex elements of block (k,q) inside M_k[k]
  int64_t ws_off;          // complex elements of the pair's sparse block inside the workspace
  int64_t u_off;           // lds_t elements of plane 0 of q inside the prepared factor
  int32_t ldu;             // padded order of the factor of q (multiple of 128)
  int32_t ldw;             // column length of the sparse workspace block
};
// One work item: pair (k,q); n'' values [g0, g1) processed ngc at a time (each
// chunk is one pass of the K loop over ngc * n_b columns); row blocks [rb0, rb1)
// of the pair (sparse row blocks first, then dense); partial slot `slot`.
struct WorkItem { int32_t pair, g0, g1, ngc, rb0, rb1, slot, pad; };

struct TileArgs {
  const PairInfo* pairs;
  const WorkItem* items;
  int32_t n_items;
  int32_t* counter;              // non-null: persistent mode (atomic work counter)
  const void* const* mtab;       // [n_k] device pointers to M_k
  int32_t m_c64;                 // 1: M holds complex64
  int32_t n_s, n_ch;
  const void* U;                 // prepared factor planes
  const void* ws;                // sparse workspace (complex, double2 or float2)
  void* gpart;                   // Gram-tile partials, acc_t
  double* dpart;                 // FP64 diagonal partials
  int32_t gstride, dstride;      // elements per slot
};

// tile pair index tp <-> (I, J), I <= J, column-wise upper triangle: tp = J(J+1)/2 + I
__device__ __forceinline__ void tp_to_ij(int tp, int& I, int& J) {
  int j = 0;
  while ((j + 1) * (j + 2) / 2 <= tp) ++j;
  J = j;
  I = tp - j * (j + 1) / 2;
}

template <int MODE, int FORM, int BM, int KC, int NCT, int NB8M>
struct TileCfg {
  using T = Traits<MODE>;
  using acc_t = typename T::acc_t;
  using lds_t = typename T::lds_t;
  using accv_t = typename T::accv_t;
  static constexpr int NP = T::NPIECE, KS = T::KS, KPL = KS / 4;   // k values each of the 4 lane groups supplies
  static constexpr int BMW = BM / 4, RT = BMW / 16;
  static constexpr int NCC = NCT * 8;
  static constexpr int PADE = 16 / (int)sizeof(lds_t);
  static constexpr int LDK = KC + PADE;
  static constexpr int LDR = BM + PADE;
  static constexpr int US_SZ = 2 * NP * BM * LDK;
  static constexpr int AS_SZ = 2 * NP * NCC * LDK;
  static constexpr int YPL = NB8M * 8 * LDR;              // one plane of the group stage
  static constexpr int YS_SZ = 2 * NP * YPL;
  static constexpr int LPL = NB8M * 8 * (BM + 2);         // GEMM left operand (double)
  static constexpr int LS_SZ = (FORM == 0) ? 2 * LPL : 0;
  static constexpr int NPT = NB8M * (NB8M + 1) / 2;
  static constexpr int NPW = (NPT + 3) / 4;
  static constexpr size_t KLOOP_B = (size_t)(US_SZ + AS_SZ) * sizeof(lds_t);
  static constexpr size_t STAGE_B = ((size_t)YS_SZ * sizeof(lds_t) + 15) / 16 * 16 + (size_t)LS_SZ * 8;
  static constexpr size_t DIAG_B = (size_t)4 * NCC * sizeof(double);
  static constexpr size_t LDS_B = KLOOP_B > STAGE_B ? (KLOOP_B > DIAG_B ? KLOOP_B : DIAG_B)
                                                    : (STAGE_B > DIAG_B ? STAGE_B : DIAG_B);
  // per-thread prefetch counts (16-byte units for U; k-pairs for A)
  static constexpr int UV_PER_PLANE = BM * KC * (int)sizeof(lds_t) / 16;
  static constexpr int UV_TOTAL = 2 * NP * UV_PER_PLANE;
  static constexpr int UV_PT = (UV_TOTAL + 255) / 256;
  static constexpr int AV_TOTAL = NCC * KC / 2;
  static constexpr int AV_PT = (AV_TOTAL + 255) / 256;
};

// Load the operand a lane supplies for one MFMA from an LDS row (k contiguous).
template <int MODE>
__device__ __forceinline__ auto lds_operand(const typename Traits<MODE>::lds_t* p) {
  if constexpr (MODE == M_F64 || MODE == M_F32) {
    return *p;
  } else {
    return *(const u4_t*)p;
  }
}

template <int MODE, int FORM, int BM, int KC, int NCT, int NB8M>
__global__ __launch_bounds__(256, 1) void tile_kernel(TileArgs a) {
  using C = TileCfg<MODE, FORM, BM, KC, NCT, NB8M>;
  using acc_t = typename C::acc_t;
  using lds_t = typename C::lds_t;
  using accv_t = typename C::accv_t;
  constexpr int NP = C::NP, KS = C::KS, KPL = C::KPL, RT = C::RT, BMW = C::BMW;
  constexpr int LDK = C::LDK, LDR = C::LDR, YPL = C::YPL;
  constexpr bool HERK = (FORM == 1);
  constexpr bool DIAG64 = HERK && (MODE != M_F64);

  __shared__ __align__(16) unsigned char smem[C::LDS_B];
  __shared__ int s_item;
  lds_t* Us = (lds_t*)smem;
  lds_t* As = Us + C::US_SZ;
  lds_t* Ys = (lds_t*)smem;
  double* Ls = (double*)(smem + ((size_t)C::YS_SZ * sizeof(lds_t) + 15) / 16 * 16);
  double* Dsum = (double*)smem;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, lq = lane >> 4;       // MFMA row/col within tile, k group
  const int c8 = l16 & 7, part = l16 >> 3;         // complex column within tile, re/im

  for (int iter = 0;; ++iter) {
    int idx;
    if (a.counter) {
      if (tid == 0) s_item = atomicAdd(a.counter, 1);
      __syncthreads();
      idx = s_item;
      __syncthreads();
    } else {
      if (iter > 0) break;
      idx = blockIdx.x;
    }
    if (idx >= a.n_items) break;

    const WorkItem wi = a.items[idx];
    const PairInfo pi = a.pairs[wi.pair];
    const int nb = pi.nb, nb8 = pi.nb8, nbt = nb8 >> 3;
    const int npt = nbt * (nbt + 1) / 2;
    const int nd = pi.nd;
    const int esz = a.m_c64 ? 8 : 16;
    const char* mbase = (const char*)a.mtab[pi.k] + pi.m_off * esz;

    accv_t gacc[C::NPW];
#pragma unroll
    for (int s = 0; s < C::NPW; ++s) gacc[s] = accv_t{0, 0, 0, 0};
    double dacc[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) dacc[t] = 0.0;

    for (int gbase = wi.g0; gbase < wi.g1; gbase += wi.ngc) {
    const int ng = min(wi.ngc, wi.g1 - gbase);
    const int nct = ng * nbt;
    const int ncols = ng * nb8;
    for (int rb = wi.rb0; rb < wi.rb1; ++rb) {
      const bool sparse = rb < pi.nsb;
      const int r0 = sparse ? rb * BM : (rb - pi.nsb) * BM;  // first row (sparse or dense coords)

      accv_t yacc[RT][NCT];
      if (!sparse) {
        // ---------------- dense rows: K loop on MFMA ----------------
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) yacc[rt][ct] = accv_t{0, 0, 0, 0};
        const int kc0 = HERK ? (r0 / KC) * KC : 0;
        const int kc1 = (nd + KC - 1) / KC * KC;
        const lds_t* Ug = (const lds_t*)a.U + pi.u_off;
        const long plane = (long)pi.ldu * pi.ldu;

        u4_t ureg[C::UV_PT];
        u4_t areg[C::AV_PT][2];
        auto prefetch = [&](int kc) {
#pragma unroll
          for (int j = 0; j < C::UV_PT; ++j) {
            const int v = tid + 256 * j;
            if (v < C::UV_TOTAL) {
              const int pl = v / C::UV_PER_PLANE, rem = v % C::UV_PER_PLANE;
              constexpr int VPR = KC * (int)sizeof(lds_t) / 16;   // 16-byte vectors per row
              const int row = rem / VPR, kv = rem % VPR;
              const lds_t* src = Ug + pl * plane + (long)(r0 + row) * pi.ldu + kc + kv * (16 / (int)sizeof(lds_t));
              ureg[j] = *(const u4_t*)src;
            }
          }
#pragma unroll
          for (int j = 0; j < C::AV_PT; ++j) {
            const int v = tid + 256 * j;
            areg[j][0] = u4_t{0, 0, 0, 0};
            areg[j][1] = u4_t{0, 0, 0, 0};
            if (v < C::AV_TOTAL) {
              const int c = v / (KC / 2), kp = v % (KC / 2);
              const int g = c / nb8, n = c - g * nb8;
              const int kk = kc + 2 * kp;
              if (c < ncols && n < nb && kk < nd) {
                const long e = ((long)(gbase + g) * nb + n) * pi.nmb + a.n_s + kk;
                if (a.m_c64) {
                  const float* p = (const float*)mbase + 2 * e;
                  const float2 x0 = *(const float2*)p;
                  float2 x1 = make_float2(0.f, 0.f);
                  if (kk + 1 < nd) x1 = *(const float2*)(p + 2);
                  areg[j][0] = u4_t{__float_as_uint(x0.x), __float_as_uint(x0.y),
                                    __float_as_uint(x1.x), __float_as_uint(x1.y)};
                } else {
                  const u4_t* p = (const u4_t*)(mbase + 16 * e);
                  areg[j][0] = p[0];
                  if (kk + 1 < nd) areg[j][1] = p[1];
                }
              }
            }
          }
        };
        auto stage = [&]() {
#pragma unroll
          for (int j = 0; j < C::UV_PT; ++j) {
            const int v = tid + 256 * j;
            if (v < C::UV_TOTAL) {
              const int pl = v / C::UV_PER_PLANE, rem = v % C::UV_PER_PLANE;
              constexpr int VPR = KC * (int)sizeof(lds_t) / 16;
              const int row = rem / VPR, kv = rem % VPR;
              *(u4_t*)(Us + pl * (BM * LDK) + row * LDK + kv * (16 / (int)sizeof(lds_t))) = ureg[j];
            }
          }
          constexpr int APL = C::NCC * LDK;   // one plane of As
#pragma unroll
          for (int j = 0; j < C::AV_PT; ++j) {
            const int v = tid + 256 * j;
            if (v < C::AV_TOTAL) {
              const int c = v / (KC / 2), kp = v % (KC / 2);
              double re0, im0, re1, im1;
              if (a.m_c64) {
                re0 = __uint_as_float(areg[j][0].x); im0 = __uint_as_float(areg[j][0].y);
                re1 = __uint_as_float(areg[j][0].z); im1 = __uint_as_float(areg[j][0].w);
              } else {
                re0 = __hiloint2double(areg[j][0].y, areg[j][0].x);
                im0 = __hiloint2double(areg[j][0].w, areg[j][0].z);
                re1 = __hiloint2double(areg[j][1].y, areg[j][1].x);
                im1 = __hiloint2double(areg[j][1].w, areg[j][1].z);
              }
              lds_t* d = As + c * LDK + 2 * kp;
              if constexpr (MODE == M_F64) {
                *(double2*)(d) = make_double2(re0, re1);
                *(double2*)(d + NP * APL) = make_double2(im0, im1);
              } else if constexpr (MODE == M_F32) {
                *(float2*)(d) = make_float2((float)re0, (float)re1);
                *(float2*)(d + NP * APL) = make_float2((float)im0, (float)im1);
              } else {
                uint16_t h0[NP], h1[NP], g0[NP], g1[NP];
                split_d<NP>(re0, h0); split_d<NP>(re1, h1);
                split_d<NP>(im0, g0); split_d<NP>(im1, g1);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                  *(uint32_t*)(d + p * APL) = (uint32_t)h0[p] | ((uint32_t)h1[p] << 16);
                  *(uint32_t*)(d + (NP + p) * APL) = (uint32_t)g0[p] | ((uint32_t)g1[p] << 16);
                }
              }
            }
          }
        };

        prefetch(kc0);
        for (int kc = kc0; kc < kc1; kc += KC) {
          __syncthreads();
          stage();
          __syncthreads();
          if (kc + KC < kc1) prefetch(kc + KC);
#pragma unroll
          for (int ks = 0; ks < KC / KS; ++ks) {
            const int kofs = ks * KS + KPL * lq;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              decltype(lds_operand<MODE>(Us)) aop[RT][NP];
#pragma unroll
              for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                  aop[rt][p] = lds_operand<MODE>(Us + (h * NP + p) * (BM * LDK) +
                                                 (w * BMW + rt * 16 + l16) * LDK + kofs);
              const int bpart = part ^ h;
              const bool neg = (h == 1) && (part == 0);
#pragma unroll
              for (int ct = 0; ct < NCT; ++ct) {
                if (ct < nct) {
                  decltype(lds_operand<MODE>(As)) bop[NP];
#pragma unroll
                  for (int p = 0; p < NP; ++p) {
                    bop[p] = lds_operand<MODE>(As + (bpart * NP + p) * (C::NCC * LDK) + (ct * 8 + c8) * LDK + kofs);
                    if (neg) bop[p] = negate(bop[p]);
                  }
#pragma unroll
                  for (int rt = 0; rt < RT; ++rt) {
                    if constexpr (NP == 1) {
                      yacc[rt][ct] = mfma(aop[rt][0], bop[0], yacc[rt][ct]);
                    } else {
#pragma unroll
                      for (int pr = 0; pr < C::T::NPROD; ++pr)
                        yacc[rt][ct] = mfma(aop[rt][prod_a(NP, pr)], bop[prod_b(NP, pr)], yacc[rt][ct]);
                    }
                  }
                }
              }
            }
          }
        }
        if constexpr (DIAG64) {
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const double y = (double)yacc[rt][ct][i];
                dacc[ct] += y * y;
              }
        }
        if constexpr (!HERK) {
          // W rows of the multipole functions receive C_c^H A_c from the sparse kernel
          if (r0 < a.n_ch) {
            const double* X = (const double*)a.ws + 2 * pi.ws_off;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
              if (ct < nct) {
                const int c = ct * 8 + c8, g = c / nb8, n = c - g * nb8;
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                  for (int i = 0; i < 4; ++i) {
                    const int d = r0 + w * BMW + rt * 16 + acc_row<MODE>(lq, i);
                    if (d < a.n_ch && n < nb)
                      yacc[rt][ct][i] += X[2 * (((long)(gbase + g) * nb + n) * pi.ldw + a.n_s + d) + part];
                  }
              }
            }
          }
        }
      }

      // ---------------- per n'' group: stage rows, contract ----------------
      for (int g = 0; g < ng; ++g) {
        __syncthreads();
        if (!sparse) {
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            if (ct >= g * nbt && ct < (g + 1) * nbt) {
              const int cl = (ct - g * nbt) * 8 + c8;
#pragma unroll
              for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int row = w * BMW + rt * 16 + acc_row<MODE>(lq, i);
                  if constexpr (MODE == M_F64)
                    Ys[(part * NP) * YPL + cl * LDR + row] = yacc[rt][ct][i];
                  else
                    put_realf<MODE>(Ys + (part * NP) * YPL + cl * LDR + row, YPL, (float)yacc[rt][ct][i]);
                }
            }
          }
          if constexpr (!HERK) {
            // left operand: A_d rows [r0, r0+BM) of group g, FP64
            for (int e = tid; e < nb8 * BM; e += 256) {
              const int cl = e / BM, row = e - cl * BM;
              const int d = r0 + row;
              double re = 0.0, im = 0.0;
              if (cl < nb && d < nd) {
                const double* p = (const double*)(mbase + 16 * (((long)(gbase + g) * nb + cl) * pi.nmb + a.n_s + d));
                re = p[0]; im = p[1];
              }
              Ls[cl * (BM + 2) + row] = re;
              Ls[C::LPL + cl * (BM + 2) + row] = im;
            }
          }
        } else {
          // sparse rows: Y_s (HERK) or W_s (GEMM) from the workspace, A_s for GEMM
          for (int e = tid; e < nb8 * BM; e += 256) {
            const int cl = e / BM, row = e - cl * BM;
            const int r = r0 + row;
            double re = 0.0, im = 0.0;
            if (cl < nb && r < a.n_s) {
              const long wo = pi.ws_off + ((long)(gbase + g) * nb + cl) * pi.ldw + r;
              if constexpr (MODE == M_F64) {
                const double2 v = ((const double2*)a.ws)[wo];
                re = v.x; im = v.y;
              } else {
                const float2 v = ((const float2*)a.ws)[wo];
                re = v.x; im = v.y;
              }
            }
            lds_t* d = Ys + cl * LDR + row;
            if constexpr (MODE == M_F64) {
              d[0] = re; d[NP * YPL] = im;
            } else {
              put_realf<MODE>(d, YPL, (float)re);
              put_realf<MODE>(d + NP * YPL, YPL, (float)im);
            }
            if constexpr (!HERK) {
              double lre = 0.0, lim = 0.0;
              if (cl < nb && r < a.n_s) {
                const double* p = (const double*)(mbase + 16 * (((long)(gbase + g) * nb + cl) * pi.nmb + r));
                lre = p[0]; lim = p[1];
              }
              Ls[cl * (BM + 2) + row] = lre;
              Ls[C::LPL + cl * (BM + 2) + row] = lim;
            }
          }
        }
        __syncthreads();
        // contraction: this wave's Gram tiles, K = BM rows
#pragma unroll
        for (int s = 0; s < C::NPW; ++s) {
          const int tp = w + 4 * s;
          if (tp < npt) {
            int I, J;
            tp_to_ij(tp, I, J);
            const int cA = I * 8 + c8, cB = J * 8 + c8;
#pragma unroll
            for (int ks = 0; ks < BM / KS; ++ks) {
              const int kofs = ks * KS + KPL * lq;
              if constexpr (HERK) {
                decltype(lds_operand<MODE>(Ys)) ao[NP], bo[NP];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                  ao[p] = lds_operand<MODE>(Ys + (part * NP + p) * YPL + cA * LDR + kofs);
                  bo[p] = lds_operand<MODE>(Ys + (part * NP + p) * YPL + cB * LDR + kofs);
                }
                if constexpr (NP == 1) {
                  gacc[s] = mfma(ao[0], bo[0], gacc[s]);
                } else {
#pragma unroll
                  for (int pr = 0; pr < C::T::NPROD; ++pr)
                    gacc[s] = mfma(ao[prod_a(NP, pr)], bo[prod_b(NP, pr)], gacc[s]);
                }
              } else {
                const double ao = Ls[part * C::LPL + cA * (BM + 2) + kofs];
                const double bo = Ys[part * YPL + cB * LDR + kofs];
                gacc[s] = mfma(ao, bo, gacc[s]);
              }
            }
          }
        }
      }
    }

    }  // n'' chunks

    // ---------------- write the item's partials ----------------
    acc_t* gp = (acc_t*)a.gpart + (long)wi.slot * a.gstride;
#pragma unroll
    for (int s = 0; s < C::NPW; ++s) {
      const int tp = w + 4 * s;
      if (tp < npt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) gp[(tp * 4 + i) * 64 + lane] = gacc[s][i];
      }
    }
    if constexpr (DIAG64) {
      __syncthreads();
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        double d = dacc[ct];
        d += __shfl_xor(d, 16);
        d += __shfl_xor(d, 32);
        d += __shfl_xor(d, 8);
        if (lane < 8) Dsum[w * C::NCC + ct * 8 + lane] = d;
      }
      __syncthreads();
      for (int n = tid; n < nb8; n += 256) {
        double s = 0.0;
        for (int c = n; c < C::NCC; c += nb8)   // same band in every group position
          for (int ww = 0; ww < 4; ++ww) s += Dsum[ww * C::NCC + c];
        a.dpart[(long)wi.slot * a.dstride + n] = s;
      }
    }
    __syncthreads();
  }
}

}  // namespace exc
