// Fused dense tile kernel: Y = B A on MFMA for the dense rows of the mixed
// product basis, followed in the same workgroup by the contraction
// G += Left^H Right over the rows of the tile.
//
//   HERK form (v = L L^H):  B = L22^H (upper triangular), Left = Right = Y.
//   GEMM form:              B = E(q) (full), Right = W = E A_d + X, Left = A_d.
//
// The product with v(q) and the band contraction are the two stages of the
// vector-matrix-vector form (Sec. III.C, eq. "vec-mat-vec"); the dense block is
// the "one big block" of multipole functions and plane waves of Fig. 1.
//
// Complex arithmetic on real MFMA: the 16 real columns of one MFMA tile hold
// 8 complex columns, real parts in tile columns 0-7 and imaginary parts in
// 8-15. Y = B A is computed as two real products over the k index,
//   [Yr | Yi] += Br [Ar | Ai] + Bi [-Ai | Ar],
// so a complex multiply-add costs 4 real multiply-adds and odd band counts
// waste at most 7 columns.
//
// Work decomposition: the K
// loop stages row panels of B and column panels of A through NBUF LDS buffers
// (with two: one barrier per chunk; global loads for chunk i+1 are in flight
// while chunk i runs on MFMA). Wavefronts form an NWR x NWC grid over the rows
// and column tiles of a row block, so one B-operand load feeds RT row tiles.
// After the K loop the whole row block (every n'' group of the pass) is staged
// in LDS once and each wavefront contracts its own 16x16 Gram tiles G(I,J),
// I <= J, over all rows and groups.
//
// Partials: each work item (pair (k,q), a range of n'' values, a range of row
// blocks) writes its Gram tiles (plus, in the reduced-precision modes, an FP64
// sum of |Y|^2 per band) to its own slot; a separate kernel sums the slots of
// each k in a fixed order in FP64 (deterministic).
#pragma once
#include "common.hpp"

namespace exc {

struct PairInfo {
  int32_t k, q, nb, nmb;     // k, q, bands n_b(k), N_MB(q)
  int32_t nd, nsb, nb8, ndb; // N_d(q), sparse row blocks, n_b rounded to 8, dense row blocks
  int64_t m_off;             // complex elements of block (k,q) inside M_k[k]
  int64_t ws_off;            // elements (see ldw) of the pair's sparse block inside the workspace
  int64_t u_off;             // lds_t elements of plane 0 of q inside the prepared factor
  int32_t ldu;               // padded order of the factor of q (multiple of 128)
  int32_t ldw;               // row pitch of one column (one plane) of the sparse workspace
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
  int32_t n_s, n_ch, n_occ;
  int32_t ns_pad;                // reduced precision: first dense row of a packed column
  const void* U;                 // prepared factor planes
  const void* ws;                // sparse workspace: double2 (FP64) or split planes (others)
  const double* dsp;             // reduced precision: FP64 sum_r |Y_s|^2 per (pair, n'', n)
  int32_t dsp_stride;            // n_occ * nb_max
  void* gpart;                   // Gram-tile partials, acc_t
  double* dpart;                 // FP64 diagonal partials
  int32_t gstride, dstride;      // elements per slot
  const uint64_t* tmask;         // [n_k][3] band-tile pairs to compute (bit tp), nullptr: all
};

// Bit s of the result: the band mask of k keeps tile tp = w + nw s (s < ns <= 64).
// A tile pair (I, J) that is left out contributes zero to its partial slot.
__device__ __forceinline__ uint64_t tile_keep_bits(const uint64_t* tmask, int k, int w, int nw, int ns) {
  if (!tmask) return ~0ull;
  const uint64_t m0 = tmask[3 * k], m1 = tmask[3 * k + 1], m2 = tmask[3 * k + 2];
  uint64_t r = 0;
  for (int s = 0; s < ns && s < 64; ++s) {
    const int tp = w + nw * s;
    const uint64_t word = tp < 64 ? m0 : (tp < 128 ? m1 : m2);
    if (tp < 192 && ((word >> (tp & 63)) & 1)) r |= 1ull << s;
  }
  return r;
}

// tile pair index tp <-> (I, J), I <= J, column-wise upper triangle: tp = J(J+1)/2 + I
__device__ __forceinline__ void tp_to_ij(int tp, int& I, int& J) {
  int j = 0;
  while ((j + 1) * (j + 2) / 2 <= tp) ++j;
  J = j;
  I = tp - j * (j + 1) / 2;
}

template <int MODE, int FORM, int BM, int KC, int NCT, int NB8M, int NWR, int NWC, int NBUF>
struct TileCfg {
  using T = Traits<MODE>;
  using acc_t = typename T::acc_t;
  using lds_t = typename T::lds_t;
  using accv_t = typename T::accv_t;
  static constexpr int NW = NWR * NWC;                  // wavefronts: NWR along rows x NWC along columns
  static constexpr int NT = 64 * NW;                    // threads
  static constexpr int NP = T::NPIECE, KS = T::KS;
  static constexpr int KPL = KS / 4;                    // k values each of the 4 lane groups supplies
  static constexpr int BMW = BM / NWR, RT = BMW / 16;
  static_assert(RT >= 1 && BMW % 16 == 0, "each wavefront owns whole 16-row tiles");
  static constexpr int CTW = NCT / NWC;                 // column tiles per wavefront
  static_assert(CTW * NWC == NCT, "column tiles split evenly over the wavefronts");
  static constexpr int NCC = NCT * 8;
  static constexpr int PADE = 16 / (int)sizeof(lds_t);
  static constexpr int LDK = KC + PADE;
  static constexpr int LDR = BM + PADE;
  static constexpr int NPL = 2 * NP;                    // planes: re pieces, im pieces
  static constexpr int UPL = BM * LDK;                  // one plane of the B stage
  static constexpr int APL = NCC * LDK;                 // one plane of the A stage
  static constexpr int STAGE = NPL * (UPL + APL);       // lds_t elements of one K-loop buffer
  static constexpr int YPL = NCC * LDR;                 // one plane of the row-block stage (all n'' groups)
  static constexpr int YS_SZ = NPL * YPL;
  static constexpr int LPL = NCC * (BM + 2);            // GEMM left operand (double)
  static constexpr int LS_SZ = (FORM == 0) ? 2 * LPL : 0;
  static constexpr int NPT = NB8M * (NB8M + 1) / 2;
  static constexpr int NPW = (NPT + NW - 1) / NW;
  // Many Gram tiles per wave (large n_b) do not fit in registers next to the Y
  // accumulators: then each tile is accumulated for one row block at a time and
  // added into the item's private partial slot in global memory.
  static constexpr bool GSTREAM = NPW * 4 * (int)sizeof(acc_t) / 4 > 32;
  // binary32 Gram chains (for error models): one per item, or (GSTREAM) one per row block
  // added into the item's partial; rows per chunk in the block-sparse and the dense rows
  static constexpr int GCHAIN = GSTREAM ? 1 : 0, GCH_RS = BM, GCH_RD = BM;
  static constexpr size_t KLOOP_B = (size_t)NBUF * STAGE * sizeof(lds_t);
  static constexpr size_t STAGE_B = ((size_t)YS_SZ * sizeof(lds_t) + 15) / 16 * 16 + (size_t)LS_SZ * 8;
  static constexpr size_t MAIN_B = KLOOP_B > STAGE_B ? KLOOP_B : STAGE_B;
  static constexpr size_t DACC_B = (MODE != M_F64 && FORM == 1) ? (size_t)NW * NCC * 2 * sizeof(double) : 0;
  static constexpr size_t LDS_B = MAIN_B + DACC_B;
  static_assert(LDS_B + 16 <= 163840, "tile configuration exceeds the 160 KB of LDS");
  static_assert(NBUF == 1 || NBUF == 2, "one or two K-loop buffers");
  // per-thread prefetch counts (16-byte units for B; k-pairs for A)
  static constexpr int UV_PER_PLANE = BM * KC * (int)sizeof(lds_t) / 16;
  static constexpr int UV_TOTAL = NPL * UV_PER_PLANE;
  static constexpr int UV_PT = (UV_TOTAL + NT - 1) / NT;
  static constexpr int AV_TOTAL = NCC * KC / 2;
  static constexpr int AV_PT = (AV_TOTAL + NT - 1) / NT;
  // reduced precision: A comes pre-split; 16-byte vectors of k per (plane, column)
  static constexpr int EPV = 16 / (int)sizeof(lds_t);
  static constexpr int PV_PER_PLANE = NCC * KC / EPV;
  static constexpr int PV_TOTAL = NPL * PV_PER_PLANE;
  static constexpr int PV_PT = (PV_TOTAL + NT - 1) / NT;
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

template <int MODE, int FORM, int BM, int KC, int NCT, int NB8M, int NWR, int NWC, int NBUF>
__global__ __launch_bounds__(64 * NWR * NWC, 1) void tile_kernel(TileArgs a) {
  using C = TileCfg<MODE, FORM, BM, KC, NCT, NB8M, NWR, NWC, NBUF>;
  constexpr int NW = C::NW, CTW = C::CTW;
  using acc_t = typename C::acc_t;
  using lds_t = typename C::lds_t;
  using accv_t = typename C::accv_t;
  constexpr int NT = C::NT, NP = C::NP, KS = C::KS, KPL = C::KPL, RT = C::RT, BMW = C::BMW;
  constexpr int LDK = C::LDK, LDR = C::LDR, YPL = C::YPL, UPL = C::UPL, APL = C::APL;
  constexpr bool HERK = (FORM == 1);
  constexpr bool DIAG64 = HERK && (MODE != M_F64);
  constexpr int ESZ = (int)sizeof(lds_t);

  __shared__ __align__(16) unsigned char smem[C::LDS_B];
  __shared__ int s_item;
  lds_t* Ys = (lds_t*)smem;
  double* Ls = (double*)(smem + ((size_t)C::YS_SZ * sizeof(lds_t) + 15) / 16 * 16);
  double* Dacc = (double*)(smem + C::MAIN_B);   // [NW][NCC][2] per-wave diagonal sums (re, im parts)

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w % NWR, wc = w / NWR;            // wavefront's row band and column-tile band
  const int l16 = lane & 15, lq = lane >> 4;       // MFMA row/col within tile, k group
  const int c8 = l16 & 7, part = l16 >> 3;         // complex column within tile, re/im

  for (int iter = 0;; ++iter) {
    int idx;
    if (a.counter) {
      if (tid == 0) s_item = atomicAdd(a.counter, 1);
      __syncthreads();
      // uniform across the workgroup: keep the item and everything derived from it
      // in scalar registers
      idx = __builtin_amdgcn_readfirstlane(s_item);
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

    constexpr int NPWR = C::GSTREAM ? 1 : C::NPW;   // Gram tiles held in registers
    accv_t gacc[NPWR];
#pragma unroll
    for (int s = 0; s < NPWR; ++s) gacc[s] = accv_t{0, 0, 0, 0};
    acc_t* gp = (acc_t*)a.gpart + (long)wi.slot * a.gstride;
    if constexpr (C::GSTREAM) {
      for (int s = 0; s < C::NPW; ++s) {
        const int tp = w + NW * s;
        if (tp < npt)
          for (int i = 0; i < 4; ++i) gp[(tp * 4 + i) * 64 + lane] = (acc_t)0;
      }
    }
    if constexpr (DIAG64) {
      for (int e = tid; e < NW * C::NCC * 2; e += NT) Dacc[e] = 0.0;
    }
    const uint64_t wkeep = tile_keep_bits(a.tmask, pi.k, w, NW, C::NPW);

    for (int gbase = wi.g0; gbase < wi.g1; gbase += wi.ngc) {
      const int ng = min(wi.ngc, wi.g1 - gbase);
      const int nct = ng * nbt;
      const int ncols = ng * nb8;
      for (int rb = wi.rb0; rb < wi.rb1; ++rb) {
        const bool sparse = rb < pi.nsb;
        const int r0 = sparse ? rb * BM : (rb - pi.nsb) * BM;  // first row (sparse or dense coords)

        accv_t yacc[RT][CTW];
        if (!sparse) {
          // ---------------- dense rows: K loop on MFMA ----------------
#pragma unroll
          for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int j = 0; j < CTW; ++j) yacc[rt][j] = accv_t{0, 0, 0, 0};
          const int kc0 = HERK ? (r0 / KC) * KC : 0;
          const int kc1 = (nd + KC - 1) / KC * KC;
          const int nch = (kc1 - kc0) / KC;
          const lds_t* Ug = (const lds_t*)a.U + pi.u_off;
          const long plane = (long)pi.ldu * pi.ldu;

          u4_t ureg[C::UV_PT];
          constexpr int AR = (MODE == M_F64) ? C::AV_PT : C::PV_PT;
          u4_t areg0[AR], areg1[(MODE == M_F64) ? C::AV_PT : 1];
          const lds_t* Pg = (const lds_t*)a.ws + pi.ws_off;   // packed columns (reduced precision)
          auto prefetch = [&](int kc) {
#pragma unroll
            for (int j = 0; j < C::UV_PT; ++j) {
              const int v = tid + NT * j;
              if (v < C::UV_TOTAL) {
                const int pl = v / C::UV_PER_PLANE, rem = v % C::UV_PER_PLANE;
                constexpr int VPR = KC * ESZ / 16;   // 16-byte vectors per row
                const int row = rem / VPR, kv = rem % VPR;
                const lds_t* src = Ug + pl * plane + (long)(r0 + row) * pi.ldu + kc + kv * (16 / ESZ);
                ureg[j] = *(const u4_t*)src;
              }
            }
            if constexpr (MODE == M_F64) {
#pragma unroll
              for (int j = 0; j < C::AV_PT; ++j) {
                const int v = tid + NT * j;
                u4_t x0 = u4_t{0, 0, 0, 0}, x1 = u4_t{0, 0, 0, 0};
                const int c = v / (KC / 2), kp = v % (KC / 2);
                const int g = c / nb8, n = c - g * nb8;
                const int kk = kc + 2 * kp;
                if (v < C::AV_TOTAL && c < ncols && n < nb && kk < nd) {
                  const long e = ((long)(gbase + g) * nb + n) * pi.nmb + a.n_s + kk;
                  if (a.m_c64) {
                    const float* p = (const float*)mbase + 2 * e;
                    const float2 f0 = *(const float2*)p;
                    const float2 f1 = (kk + 1 < nd) ? *(const float2*)(p + 2) : make_float2(0.f, 0.f);
                    x0 = u4_t{__float_as_uint(f0.x), __float_as_uint(f0.y), __float_as_uint(f1.x), __float_as_uint(f1.y)};
                  } else {
                    const u4_t* p = (const u4_t*)(mbase + 16 * e);
                    x0 = p[0];
                    if (kk + 1 < nd) x1 = p[1];
                  }
                }
                areg0[j] = x0;
                areg1[j] = x1;
              }
            } else {
#pragma unroll
              for (int j = 0; j < C::PV_PT; ++j) {
                const int v = tid + NT * j;
                u4_t x = u4_t{0, 0, 0, 0};
                constexpr int VPK = KC / C::EPV;      // vectors per column and plane
                const int pl = v / C::PV_PER_PLANE, rem = v % C::PV_PER_PLANE;
                const int c = rem / VPK, kv = rem % VPK;
                const int g = c / nb8, n = c - g * nb8;
                if (v < C::PV_TOTAL && c < ncols && n < nb)
                  x = *(const u4_t*)(Pg + (((long)(gbase + g) * nb + n) * C::NPL + pl) * pi.ldw + a.ns_pad + kc + kv * C::EPV);
                areg0[j] = x;
              }
            }
          };
          auto stage = [&](lds_t* Us, lds_t* As) {
#pragma unroll
            for (int j = 0; j < C::UV_PT; ++j) {
              const int v = tid + NT * j;
              if (v < C::UV_TOTAL) {
                const int pl = v / C::UV_PER_PLANE, rem = v % C::UV_PER_PLANE;
                constexpr int VPR = KC * ESZ / 16;
                const int row = rem / VPR, kv = rem % VPR;
                *(u4_t*)(Us + pl * UPL + row * LDK + kv * (16 / ESZ)) = ureg[j];
              }
            }
            if constexpr (MODE == M_F64) {
#pragma unroll
              for (int j = 0; j < C::AV_PT; ++j) {
                const int v = tid + NT * j;
                if (v < C::AV_TOTAL) {
                  const int c = v / (KC / 2), kp = v % (KC / 2);
                  const u4_t x0 = areg0[j], x1 = areg1[j];
                  double re0, im0, re1, im1;
                  if (a.m_c64) {
                    re0 = __uint_as_float(x0.x); im0 = __uint_as_float(x0.y);
                    re1 = __uint_as_float(x0.z); im1 = __uint_as_float(x0.w);
                  } else {
                    re0 = __hiloint2double(x0.y, x0.x);
                    im0 = __hiloint2double(x0.w, x0.z);
                    re1 = __hiloint2double(x1.y, x1.x);
                    im1 = __hiloint2double(x1.w, x1.z);
                  }
                  lds_t* d = As + c * LDK + 2 * kp;
                  *(double2*)(d) = make_double2(re0, re1);
                  *(double2*)(d + NP * APL) = make_double2(im0, im1);
                }
              }
            } else {
#pragma unroll
              for (int j = 0; j < C::PV_PT; ++j) {
                const int v = tid + NT * j;
                if (v < C::PV_TOTAL) {
                  constexpr int VPK = KC / C::EPV;
                  const int pl = v / C::PV_PER_PLANE, rem = v % C::PV_PER_PLANE;
                  const int c = rem / VPK, kv = rem % VPK;
                  *(u4_t*)(As + pl * APL + c * LDK + kv * C::EPV) = areg0[j];
                }
              }
            }
          };

          lds_t* buf0 = (lds_t*)smem;
          lds_t* buf1 = buf0 + (NBUF == 2 ? C::STAGE : 0);
          __syncthreads();                      // previous users of the LDS are done
          prefetch(kc0);
          stage(buf0, buf0 + C::NPL * UPL);
          __syncthreads();
          for (int i = 0; i < nch; ++i) {
            lds_t* Us = (i & 1) ? buf1 : buf0;
            lds_t* As = Us + C::NPL * UPL;
            if (i + 1 < nch) prefetch(kc0 + (i + 1) * KC);
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
                    aop[rt][p] = lds_operand<MODE>(Us + (h * NP + p) * UPL + (wr * BMW + rt * 16 + l16) * LDK + kofs);
                const int bpart = part ^ h;
                const bool neg = (h == 1) && (part == 0);
                // this wave's CTW column tiles: columns beyond the item are zero in LDS
#pragma unroll
                for (int j = 0; j < CTW; ++j) {
                  const int ct = wc * CTW + j;
                  decltype(lds_operand<MODE>(As)) bop[NP];
#pragma unroll
                  for (int p = 0; p < NP; ++p) {
                    bop[p] = lds_operand<MODE>(As + (bpart * NP + p) * APL + (ct * 8 + c8) * LDK + kofs);
                    if (neg) bop[p] = negate(bop[p]);
                  }
#pragma unroll
                  for (int rt = 0; rt < RT; ++rt) {
                    if constexpr (NP == 1) {
                      yacc[rt][j] = mfma(aop[rt][0], bop[0], yacc[rt][j]);
                    } else {
#pragma unroll
                      for (int pr = 0; pr < C::T::NPROD; ++pr)
                        yacc[rt][j] = mfma(aop[rt][prod_a(NP, pr)], bop[prod_b(NP, pr)], yacc[rt][j]);
                    }
                  }
                }
              }
            }
            if (i + 1 < nch) {
              if constexpr (NBUF == 1) __syncthreads();   // every wave is done with the only buffer
              stage((i & 1) ? buf0 : buf1, ((i & 1) ? buf0 : buf1) + C::NPL * UPL);
            }
            __syncthreads();
          }
          if constexpr (DIAG64) {
            // FP64 sums of |Y|^2 per real column; the four lanes of one column are
            // reduced first so that each wave owns its Dacc row (no races, fixed order)
#pragma unroll
            for (int j = 0; j < CTW; ++j) {
              const int ct = wc * CTW + j;
              double d = 0.0;
#pragma unroll
              for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const double y = (double)yacc[rt][j][i];
                  d += y * y;
                }
              d += __shfl_xor(d, 16);
              d += __shfl_xor(d, 32);
              if (lq == 0) Dacc[(w * C::NCC + ct * 8 + c8) * 2 + part] += d;
            }
          }
          if constexpr (!HERK) {
            // W rows of the multipole functions receive C_c^H A_c from the sparse kernel
            if (r0 < a.n_ch) {
              const double* X = (const double*)a.ws + 2 * pi.ws_off;
#pragma unroll
              for (int j = 0; j < CTW; ++j) {
                const int ct = wc * CTW + j;
                if (ct < nct) {
                  const int c = ct * 8 + c8, g = c / nb8, n = c - g * nb8;
#pragma unroll
                  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                      const int d = r0 + wr * BMW + rt * 16 + acc_row<MODE>(lq, i);
                      if (d < a.n_ch && n < nb)
                        yacc[rt][j][i] += X[2 * (((long)(gbase + g) * nb + n) * pi.ldw + a.n_s + d) + part];
                    }
                }
              }
            }
          }
        }

        // ---------------- stage the row block (all n'' groups), contract ----------------
        __syncthreads();
        if (!sparse) {
#pragma unroll
          for (int j = 0; j < CTW; ++j) {
            const int cl = (wc * CTW + j) * 8 + c8;   // column within the pass (group-major)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int row = wr * BMW + rt * 16 + acc_row<MODE>(lq, i);
                if constexpr (MODE == M_F64)
                  Ys[(part * NP) * YPL + cl * LDR + row] = yacc[rt][j][i];
                else
                  put_realf<MODE>(Ys + (part * NP) * YPL + cl * LDR + row, YPL, (float)yacc[rt][j][i]);
              }
          }
          if constexpr (!HERK) {
            // left operand: A_d rows [r0, r0+BM) of every group of the pass, FP64
            for (int e = tid; e < ncols * BM; e += NT) {
              const int cl = e / BM, row = e - cl * BM;
              const int g = cl / nb8, n = cl - g * nb8;
              const int d = r0 + row;
              double re = 0.0, im = 0.0;
              if (n < nb && d < nd) {
                const double* p = (const double*)(mbase + 16 * (((long)(gbase + g) * nb + n) * pi.nmb + a.n_s + d));
                re = p[0]; im = p[1];
              }
              Ls[cl * (BM + 2) + row] = re;
              Ls[C::LPL + cl * (BM + 2) + row] = im;
            }
          }
        } else if constexpr (MODE == M_F64) {
          // sparse rows: Y_s (HERK) or W_s (GEMM) as double2 from the workspace, A_s for GEMM
          for (int e = tid; e < ncols * BM; e += NT) {
            const int cl = e / BM, row = e - cl * BM;
            const int g = cl / nb8, n = cl - g * nb8;
            const int r = r0 + row;
            double re = 0.0, im = 0.0;
            if (n < nb && r < a.n_s) {
              const double2 v = ((const double2*)a.ws)[pi.ws_off + ((long)(gbase + g) * nb + n) * pi.ldw + r];
              re = v.x; im = v.y;
            }
            Ys[cl * LDR + row] = re;
            Ys[YPL + cl * LDR + row] = im;
            if constexpr (!HERK) {
              double lre = 0.0, lim = 0.0;
              if (n < nb && r < a.n_s) {
                const double* p = (const double*)(mbase + 16 * (((long)(gbase + g) * nb + n) * pi.nmb + r));
                lre = p[0]; lim = p[1];
              }
              Ls[cl * (BM + 2) + row] = lre;
              Ls[C::LPL + cl * (BM + 2) + row] = lim;
            }
          }
        } else {
          // sparse rows, reduced precision: the block-sparse kernel wrote Y_s already split
          // into planes [n''][n][plane][row] (pitch ldw, zero padded to ns_pad rows): 16-byte copies
          constexpr int EPV = 16 / ESZ;                       // elements per 16-byte vector
          constexpr int VPC = BM / EPV;                       // vectors per column and plane
          const lds_t* src = (const lds_t*)a.ws + pi.ws_off;
          for (int v = tid; v < C::NPL * ncols * VPC; v += NT) {
            const int pl = v / (ncols * VPC), rem = v - pl * (ncols * VPC);
            const int cl = rem / VPC, rv = rem - cl * VPC;
            const int g = cl / nb8, n = cl - g * nb8;
            const int r = r0 + rv * EPV;
            u4_t x = u4_t{0, 0, 0, 0};
            if (n < nb && r < a.ns_pad)
              x = *(const u4_t*)(src + (((long)(gbase + g) * nb + n) * C::NPL + pl) * pi.ldw + r);
            *(u4_t*)(Ys + pl * YPL + cl * LDR + rv * EPV) = x;
          }
        }
        __syncthreads();
        // contraction: this wave's Gram tiles over the BM rows of every group of the pass
        auto contract = [&](int tp, int g, accv_t acc) -> accv_t {
          int I, J;
          tp_to_ij(tp, I, J);
          const int cA = g * nb8 + I * 8 + c8, cB = g * nb8 + J * 8 + c8;
#pragma unroll 2
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
                acc = mfma(ao[0], bo[0], acc);
              } else {
#pragma unroll
                for (int pr = 0; pr < C::T::NPROD; ++pr)
                  acc = mfma(ao[prod_a(NP, pr)], bo[prod_b(NP, pr)], acc);
              }
            } else {
              const double ao = Ls[part * C::LPL + cA * (BM + 2) + kofs];
              const double bo = Ys[part * YPL + cB * LDR + kofs];
              acc = mfma(ao, bo, acc);
            }
          }
          return acc;
        };
        if constexpr (C::GSTREAM) {
          for (int s = 0; s < C::NPW; ++s) {
            const int tp = w + NW * s;
            if (tp >= npt) break;
            if (!((wkeep >> s) & 1)) continue;
            accv_t acc = accv_t{0, 0, 0, 0};
            for (int g = 0; g < ng; ++g) acc = contract(tp, g, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) gp[(tp * 4 + i) * 64 + lane] += acc[i];
          }
        } else {
#pragma unroll
          for (int s = 0; s < NPWR; ++s) {
            const int tp = w + NW * s;
            if (tp < npt && ((wkeep >> s) & 1))
              for (int g = 0; g < ng; ++g) gacc[s] = contract(tp, g, gacc[s]);
          }
        }
      }
    }  // n'' chunks

    // ---------------- write the item's partials ----------------
    if constexpr (!C::GSTREAM) {
#pragma unroll
      for (int s = 0; s < NPWR; ++s) {
        const int tp = w + NW * s;
        if (tp < npt) {
#pragma unroll
          for (int i = 0; i < 4; ++i) gp[(tp * 4 + i) * 64 + lane] = gacc[s][i];
        }
      }
    }
    if constexpr (DIAG64) {
      __syncthreads();
      for (int n = tid; n < nb8; n += NT) {
        double s = 0.0;
        for (int c = n; c < C::NCC; c += nb8)   // same band in every group position
          for (int ww = 0; ww < NW; ++ww) s += Dacc[(ww * C::NCC + c) * 2] + Dacc[(ww * C::NCC + c) * 2 + 1];
        // multipole-free rows: FP64 sums from the block-sparse kernel, added once per
        // (pair, n'') by the item that holds the pair's first row block
        if (wi.rb0 == 0 && n < nb)
          for (int j = wi.g0; j < wi.g1; ++j) s += a.dsp[(long)wi.pair * a.dsp_stride + (long)j * nb + n];
        a.dpart[(long)wi.slot * a.dstride + n] = s;
      }
    }
    __syncthreads();
  }
}

}  // namespace exc
