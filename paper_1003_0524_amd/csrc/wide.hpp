// Wide exchange kernel for large (k, q) pairs in the reduced-precision Cholesky/HERK
// form (complex64 M): the same work item and partial layout as fused_kernel -- a
// pair and a range of n'' values, G = sum_{n''} Y^H Y with Y = [Y_s ; Y_d],
// Y_s = L_c^H A_c + l_c a_{j(c)} (block-sparse rows, FP64 VALU) and Y_d = L22^H A_d
// (dense rows, MFMA in the mode's pieces) -- laid out for mixed bases of thousands
// of functions and 50-128 bands (Sec. III.C, eq. "vec-mat-vec"; Fig. 1 sparsity):
//
//  * 8 wavefronts (two per SIMD), one workgroup per CU: while one wavefront of a
//    SIMD waits at a barrier or on memory the other issues matrix instructions;
//  * dense row blocks of 256 rows (two 16-row tiles per wavefront), so each K panel
//    of A_d is read and converted once for 256 rows of the factor;
//  * K panels of A_d move global -> LDS by direct buffer loads three panels ahead
//    (complex64: 26 KB a panel), are split into bf16 / FP32 pieces once per panel
//    (binary32 arithmetic: complex64 inputs split exactly as from their float64
//    value), into one of two piece buffers: one workgroup barrier per panel;
//  * the factor pieces of the wavefront's rows come from L2 one panel ahead;
//  * the Gram tiles of an n'' chunk stay in registers (at most 17 per wavefront) and
//    go to the item's partial slot once per chunk (not once per 64 rows).
// The block-sparse phase takes fused_kernel's chunks of whole channels, with one
// column per lane and each row's run of the triangle exactly (no padding to the
// chunk's longest run), the chunk's values of M staged in LDS.
#pragma once
#include "fused.hpp"

#include <utility>

namespace exc {


// Gram tile schedule of the wide kernel: the upper triangle of NCT x NCT band tiles is split into
// units -- a row pair m (band tiles 2m, 2m + 1) times a band-tile range [j0, j1) -- at most two per
// wavefront. Per 32 rows a unit reads its two row operands once and each column operand once for both
// rows, where the round robin (tile w + 8 s) reads both operands of every tile. The units were found by
// a search over segmentations of the row pairs' ranges, assigned longest first to the least loaded
// wavefront: 12 tiles per wavefront for 13 band tiles (17 for 16), as many as the round robin, with at
// most 10 (13) operand reads per 32 rows instead of 24 (34).
struct GramUnits { int u[8][2][3]; };
constexpr GramUnits gram_units(int nct) {
  return nct == 13 ? GramUnits{{{{0, 6, 12}, {-1, 0, 0}}, {{0, 0, 6}, {6, 12, 13}}, {{1, 2, 8}, {-1, 0, 0}},
                                {{2, 4, 10}, {-1, 0, 0}}, {{3, 6, 12}, {-1, 0, 0}}, {{1, 8, 13}, {3, 12, 13}},
                                {{4, 8, 13}, {0, 12, 13}}, {{2, 10, 13}, {5, 10, 13}}}}
                   : GramUnits{{{{0, 0, 9}, {-1, 0, 0}}, {{1, 2, 11}, {-1, 0, 0}}, {{2, 4, 13}, {-1, 0, 0}},
                                {{3, 6, 15}, {-1, 0, 0}}, {{4, 8, 16}, {3, 15, 16}}, {{0, 9, 16}, {7, 14, 16}},
                                {{5, 10, 16}, {2, 13, 16}}, {{1, 11, 16}, {6, 12, 16}}}};
}
template <int NCT>
struct GramSched {
  static constexpr bool ON = NCT == 13 || NCT == 16;
  static constexpr GramUnits G = gram_units(NCT);
  static constexpr bool tile_ok(int r, int j) { return r < NCT && j >= r; }
  // slot of tile (row 2m + r, column j0 + jj) of unit k of wavefront w: tiles in unit order, then
  // column order, then row order
  static constexpr int slot(int w, int k, int jj, int r) {
    int s = 0;
    for (int kk = 0; kk <= k; ++kk) {
      const int m = G.u[w][kk][0];
      if (m < 0) continue;
      for (int j = G.u[w][kk][1]; j < G.u[w][kk][2]; ++j)
        for (int rr = 0; rr < 2; ++rr) {
          if (kk == k && j == G.u[w][k][1] + jj && rr == r) return s;
          if (tile_ok(2 * m + rr, j)) ++s;
        }
    }
    return -1;
  }
  struct Table { int tp[8][32]; };
  static constexpr Table table() {
    Table t{};
    for (int w = 0; w < 8; ++w) {
      for (int s = 0; s < 32; ++s) t.tp[w][s] = -1;
      int s = 0;
      for (int k = 0; k < 2; ++k) {
        const int m = G.u[w][k][0];
        if (m < 0) continue;
        for (int j = G.u[w][k][1]; j < G.u[w][k][2]; ++j)
          for (int r = 0; r < 2; ++r)
            if (tile_ok(2 * m + r, j)) t.tp[w][s++] = j * (j + 1) / 2 + 2 * m + r;   // tp = J(J+1)/2 + I
      }
    }
    return t;
  }
  static constexpr Table T = table();
};

template <int I0, class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I0 + I>{}), ...);
}
// f(integral_constant<int, i>) for i = B .. E-1
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (E > B) static_for_impl<B>(f, std::make_integer_sequence<int, E - B>{});
}

template <int MODE, int NB8M, int RTW = 2>
struct WideCfg {
  using T = Traits<MODE>;
  using lds_t = typename T::lds_t;
  static constexpr int NW = 8, NT = 512;
  static constexpr int RT = RTW;                      // 16-row tiles per wavefront of a dense row block
  static constexpr int BM = 16 * RT * NW;             // rows of a dense row block
  static constexpr int NP = T::NPIECE, KS = T::KS, KPL = KS / 4, NPL = 2 * NP;
  static constexpr int KC = 32;                       // k of a K panel
  static constexpr int NCT = NB8M, NCC = 8 * NCT;     // band tiles (8 complex columns each), columns
  static constexpr int ESZ = (int)sizeof(lds_t), EPV = 16 / ESZ;
  static constexpr int RAWP = NCC * KC * 8;           // bytes of a raw complex64 panel
  static constexpr int NI = (RAWP + 1023) / 1024;     // 1 KB direct loads per panel
  static constexpr int NIW = (NI + NW - 1) / NW;      // per wavefront (the extra ones land in a trash KB)
  static constexpr int RAW_B = NI * 1024;
  static constexpr size_t BUDGET = 163840 - 16 * 64 - 256;
  static constexpr size_t DACC_B = (size_t)NW * NCC * 2 * sizeof(double);
  // column pitch of a piece plane: KC plus a 16-byte skew, so that the operand reads of eight
  // consecutive columns meet distinct LDS banks, where two piece buffers so padded still fit
  // beside two raw panels (not for the six-product mode's wide instances)
  static constexpr bool SKEW = (size_t)2 * RAW_B + 1024 + (size_t)2 * 2 * NP * NCC * (KC + EPV) * ESZ + DACC_B <=
                               BUDGET;
  static constexpr int KCP = SKEW ? KC + EPV : KC;
  static constexpr int APL = NCC * KCP;               // one piece plane of a panel: [column][k]
  static constexpr int PCS = NPL * APL;               // one piece buffer (elements)
  // factor loads per wavefront and panel: each lane takes 8 consecutive k of a row per piece
  // plane (one 16-byte load for bf16 pieces, two for FP32)
  static constexpr int NFL = RT * 2 * (MODE == M_F32 ? 2 : NP);
  // block-sparse phase: a chunk of at most GR rows (whole channels) and its at most MPC
  // multipole rows; the chunk's M values are staged in LDS, XC columns at a time (all of the
  // item's columns where they fit beside the Gram stage), rows [GR + MPC] x columns, with an
  // odd pitch of XP complex64 values
  static constexpr int GR = 64, MPC = 16, MAXT = 12, MAXCK = 64;
  static constexpr int LDRS = GR + EPV;
  static constexpr size_t SS_B = (size_t)NPL * NCC * LDRS * ESZ;        // Gram stage of a chunk
  static constexpr size_t SP_TAB = (size_t)MAXT * GR * 16 + 2 * GR * 16 + 256;   // coefficients, row info, l_c, row groups
  static constexpr size_t xstage_b(int xc) { return ((size_t)(GR + MPC) * (xc + 1) * 8 + 15) / 16 * 16; }
  static constexpr int XC = SP_TAB + xstage_b(NCC) + SS_B + DACC_B <= BUDGET ? NCC : 64;
  static constexpr int XP = XC + 1;
  static constexpr int NU = (XC + 63) / 64;          // 64-column groups of a stage (one column a lane)
  static constexpr int NSTG = (NCC + XC - 1) / XC;   // stages of a chunk (at most)
  static constexpr int NDR = (NCC + 63) / 64;        // FP64 |Y|^2 sums per lane
  static constexpr int XLD = (XC * GR + NT - 1) / NT, XLM = (XC * MPC + NT - 1) / NT;   // loads per thread
  static constexpr int SP_CF = 0, SP_RI = SP_CF + MAXT * GR * 16, SP_CV = SP_RI + GR * 16, SP_GT = SP_CV + GR * 16;
  static constexpr int SP_X = SP_GT + 256;
  static constexpr size_t SP_ST = (size_t)SP_X + xstage_b(XC);
  static constexpr size_t SPARSE_B = SP_ST + SS_B;
  static_assert(MAXCK == 64, "the LDS budget above reserves 64 chunk descriptors");
  static_assert(XC % NW == 0 && (XC == NCC || XC % 64 == 0), "whole columns per wavefront; 64-column stages");
  static_assert(NDR <= 2 && NSTG <= 2, "at most two 64-column groups of a chunk");
  // Gram stage of the dense rows: GS rows at a time (rows contiguous per column)
  static constexpr int GS = (BM >= 128 && (size_t)NPL * NCC * (128 + EPV) * ESZ + DACC_B <= BUDGET) ? 128 : 64;
  static constexpr int LDR = GS + EPV;
  static constexpr size_t STAGE_B = (size_t)NPL * NCC * LDR * ESZ;
  static constexpr size_t PIECE_B = (size_t)2 * PCS * ESZ;
  static constexpr int NRAW = ((size_t)3 * RAW_B + 1024 + PIECE_B + DACC_B <= BUDGET) ? 3 : 2;
  static constexpr size_t KLOOP_B = (size_t)NRAW * RAW_B + 1024 + PIECE_B;
  static constexpr size_t M1 = KLOOP_B > STAGE_B ? KLOOP_B : STAGE_B;
  static constexpr size_t M2 = M1 > SPARSE_B ? M1 : SPARSE_B;
  static constexpr size_t MAIN_B = (M2 + 15) / 16 * 16;
  static constexpr size_t LDS_B = MAIN_B + DACC_B;
  static constexpr int NPT = NB8M * (NB8M + 1) / 2;
  static constexpr int NPW = (NPT + NW - 1) / NW;     // Gram tiles per wavefront (round robin)
  // binary32 Gram chains (for error models): one per n'' chunk, added into the item's
  // partial; GR rows per chunk in the block-sparse rows, GS in the dense rows
  static constexpr int GCHAIN = 2, GCH_RS = GR, GCH_RD = GS;
  static_assert(MODE != M_F64, "the wide kernel serves the reduced-precision modes");
  static_assert(LDS_B <= BUDGET, "wide configuration exceeds the 160 KB of LDS");
  static_assert((size_t)2 * RAW_B + 1024 + PIECE_B + DACC_B <= BUDGET, "at least two raw panels in flight");
  static_assert(KC == 32 && GS % KS == 0 && GR % KS == 0, "whole MFMA steps; 8 k per lane a panel");
  static_assert(NCC * (KC / 8) <= NT, "one conversion unit per thread and panel");
};

// vmcnt(n) alone (gfx9 encoding: expcnt and lgkmcnt at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit count");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | 0x0F70);
}

// Split 4 consecutive k of one value into the mode's pieces and store each piece
// plane's 4 values (8 B for bf16, 16 B for FP32) at dst + plane * ps.
template <int MODE>
__device__ __forceinline__ void store_pieces4(typename Traits<MODE>::lds_t* dst, int ps, float x0, float x1,
                                              float x2, float x3) {
  if constexpr (MODE == M_F32) {
    *(f4_t*)dst = f4_t{x0, x1, x2, x3};
  } else {
    constexpr int NP = Traits<MODE>::NPIECE;
    uint16_t h0[NP], h1[NP], h2[NP], h3[NP];
    split_f<NP>(x0, h0);
    split_f<NP>(x1, h1);
    split_f<NP>(x2, h2);
    split_f<NP>(x3, h3);
#pragma unroll
    for (int p = 0; p < NP; ++p)
      *(uint2*)(dst + (long)p * ps) = make_uint2((uint32_t)h0[p] | ((uint32_t)h1[p] << 16),
                                                 (uint32_t)h2[p] | ((uint32_t)h3[p] << 16));
  }
}

template <int MODE, int NB8M, int RTW>
__global__ __launch_bounds__(512, 1) void wide_kernel(FusedArgs a) {
  using C = WideCfg<MODE, NB8M, RTW>;
  using lds_t = typename C::lds_t;
  using acc_t = typename Traits<MODE>::acc_t;
  using accv_t = typename Traits<MODE>::accv_t;
  using op_t = decltype(lds_operand<MODE>((const lds_t*)nullptr));
  constexpr int NW = C::NW, NT = C::NT, NP = C::NP, KS = C::KS, KPL = C::KPL, NPL = C::NPL;
  constexpr int NCC = C::NCC, NCT = C::NCT, KC = C::KC, KCP = C::KCP, APL = C::APL, PCS = C::PCS, RT = C::RT;
  constexpr int BM = C::BM, GR = C::GR, GS = C::GS, LDR = C::LDR, NIW = C::NIW, NI = C::NI;
  constexpr int NRAW = C::NRAW, NFL = C::NFL;

  __shared__ __align__(16) unsigned char smem[C::LDS_B];
  __shared__ int s_item;
  __shared__ int4 s_chunk[C::MAXCK];
  __shared__ int s_left[NQ_MAX];
  unsigned char* Raw = smem;                                        // NRAW x [NCC][KC] complex64
  unsigned char* Trash = smem + NRAW * C::RAW_B;                    // 1 KB for the padding loads
  lds_t* Pcs = (lds_t*)(smem + NRAW * C::RAW_B + 1024);             // 2 x [NPL][NCC][KC] pieces
  lds_t* Ys = (lds_t*)smem;                                         // [NPL][NCC][LDR] Gram stage
  double* Dacc = (double*)(smem + C::MAIN_B);                       // [NW][NCC][2]

  const int tid0 = threadIdx.x;
  const int nq = a.counter ? a.nq : 1;
  const int G = (int)gridDim.x;
  const int qi = a.counter ? (int)(blockIdx.x % nq) : 0;
  auto n_static = [&](int q) { return (G - q + nq - 1) / nq; };
  int qh0 = 0, qh1 = 0;
  int idx;
  if (a.counter) {
    qh0 = uni(a.qbeg[qi]);
    qh1 = uni(a.qbeg[qi + 1]);
    const int j = qh0 + (int)blockIdx.x / nq;
    idx = j < qh1 ? j : -1;
  } else {
    idx = (int)blockIdx.x < a.n_items ? (int)blockIdx.x : -1;
  }
  bool home = a.counter != nullptr;
  auto steal = [&]() -> int {
    if (tid0 < nq) {
      const int cnt = __hip_atomic_load(a.counter + tid0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_left[tid0] = a.qbeg[tid0] + n_static(tid0) + cnt < a.qbeg[tid0 + 1];
    }
    __syncthreads();
    int got = -1;
    for (int o = 1; o < nq && got < 0; ++o) {
      const int q = (qi + o) % nq;
      if (!s_left[q]) continue;
      if (tid0 == 0) s_item = atomicAdd(a.counter + q, 1);
      __syncthreads();
      const int j = a.qbeg[q] + n_static(q) + __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();
      if (j < a.qbeg[q + 1]) got = j;
    }
    __syncthreads();
    return uni(got);
  };

  for (;;) {
    if (idx < 0) {
      if (!a.counter) break;
      idx = steal();
      if (idx < 0) break;
    }
    int claim = 0;
    if (home && tid0 == 0) claim = atomicAdd(a.counter + qi, 1);

    int tid_o = tid0;
    asm volatile("" : "+v"(tid_o));
    const int tid = tid_o, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l16 = lane & 15, lq = lane >> 4;
    const int c8 = l16 & 7, part = l16 >> 3;

    WorkItem wi = a.items[idx];
    wi.pair = uni(wi.pair); wi.g0 = uni(wi.g0); wi.g1 = uni(wi.g1); wi.ngc = uni(wi.ngc); wi.slot = uni(wi.slot);
    wi.rb0 = uni(wi.rb0); wi.rb1 = uni(wi.rb1);
    PairInfo pi = a.pairs[wi.pair];
    pi.k = uni(pi.k); pi.nb = uni(pi.nb); pi.nmb = uni(pi.nmb); pi.nd = uni(pi.nd); pi.nb8 = uni(pi.nb8);
    pi.m_off = uni(pi.m_off); pi.u_off = uni(pi.u_off); pi.ldu = uni(pi.ldu);
    const int nb = pi.nb, nb8 = pi.nb8, nbt = nb8 >> 3;
    const uint32_t nb8_rcp = uni((int32_t)(0xFFFFFFFFu / (uint32_t)nb8 + 1u));
    const int npt = nbt * (nbt + 1) / 2;
    const int nd = pi.nd;
    constexpr int esz = 8;                                          // complex64 M
    const char* mbase = uni((const char*)a.mtab[pi.k]) + pi.m_off * esz;
    const __amdgpu_buffer_rsrc_t mrs = make_rsrc(mbase, (uint32_t)((long)a.n_occ * nb * pi.nmb * esz));
    const lds_t* Ug = (const lds_t*)a.U + pi.u_off;
    const long plane = (long)pi.ldu * pi.ldu;
    const __amdgpu_buffer_rsrc_t urs = make_rsrc(Ug, (uint32_t)(NPL * plane * C::ESZ));
    const uint32_t u_lane = (uint32_t)((l16 * pi.ldu + 8 * lq) * C::ESZ);

    accv_t gacc[C::NPW];
#pragma unroll
    for (int s = 0; s < C::NPW; ++s) gacc[s] = accv_t{0, 0, 0, 0};
    acc_t* gp = (acc_t*)a.gpart + (long)wi.slot * a.gstride;
    for (int e = tid; e < NW * NCC * 2; e += NT) Dacc[e] = 0.0;
    using GU = GramSched<NCT>;
    // the unit schedule of the Gram tiles (else the round robin): measured faster for the fp32
    // instances (SrTiO3-like step 756 -> 669 ms) and for bf16x3 (262 -> 258 ms); the six-product
    // mode keeps one tile's operands at a time
    constexpr bool UNITS = GU::ON && MODE != M_BF16X6 && C::NPW <= 32;
    // tile of this wavefront's Gram slot s (band-tile pair index tp = J(J+1)/2 + I; -1: none)
    auto slot_tp = [&](int s) -> int {
      if constexpr (UNITS) return GU::T.tp[w][s];
      else return w + NW * s;
    };
    uint64_t wkeep = 0;
    if constexpr (UNITS) {
#pragma unroll
      for (int s2 = 0; s2 < C::NPW; ++s2) {
        const int tp = slot_tp(s2);
        bool keep = tp >= 0 && tp < npt;
        if (keep && a.tmask) keep = (a.tmask[3 * pi.k + (tp >> 6)] >> (tp & 63)) & 1;
        if (keep) wkeep |= 1ull << s2;
      }
    } else {
      wkeep = tile_keep_bits(a.tmask, pi.k, w, NW, C::NPW);
#pragma unroll
      for (int s2 = 0; s2 < C::NPW; ++s2)
        if (w + NW * s2 >= npt) wkeep &= ~(1ull << s2);
    }

    // ---- contraction of ROWS staged rows (pitch `pitch`) into this wave's Gram tiles ----
    // use_units (with UNITS): the unit schedule's operand reuse; else tile by tile in the same
    // slot order
    auto contract = [&](const lds_t* S, int ng, auto rows_c, int pitch, auto use_units) {
      constexpr int ROWS = decltype(rows_c)::value;
      // lane-derived addresses from an opaque copy of the lane index: formed afresh per call
      // instead of being hoisted out of the row-block loops and kept live (or spilled)
      int lx = lane;
      asm volatile("" : "+v"(lx));
      const lds_t* Sl = S + (((lx >> 3) & 1) * NP) * NCC * pitch + (lx & 7) * pitch + KPL * (lx >> 4);
      constexpr int KSN = ROWS / KS;
      static_assert(KSN % 2 == 0, "steps in pairs");
      // the operands of each (tile, step) are requested one step ahead, across tiles too: the
      // last step of a tile requests the first of the next (a tile past the triangle or masked
      // out reads band tile 0 and skips its products)
      auto bases = [&](int s, int g, const lds_t*& A_, const lds_t*& B_) {
        const int tp = slot_tp(s);
        int I = 0, J = 0;
        if (tp >= 0 && tp < npt) tp_to_ij(tp, I, J);
        A_ = Sl + (g * nb8 + I * 8) * pitch;
        B_ = Sl + (g * nb8 + J * 8) * pitch;
      };
      auto ld = [&](const lds_t* A_, const lds_t* B_, int ks, op_t (&a_)[NP], op_t (&b_)[NP]) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          a_[p] = lds_operand<MODE>(A_ + p * NCC * pitch + ks * KS);
          b_[p] = lds_operand<MODE>(B_ + p * NCC * pitch + ks * KS);
        }
      };
      if constexpr (UNITS && decltype(use_units)::value) {
        // per 32 rows: each unit's two row operands once, each column operand once for both rows
        // (the next column's requested before this one's products)
        auto run = [&](auto wc) {
          constexpr int W = decltype(wc)::value;
          for (int g = 0; g < ng; ++g) {
            const lds_t* Sg = Sl + g * nb8 * pitch;
#pragma unroll 1
            for (int ks = 0; ks < KSN; ++ks) {
              auto opnd = [&](int bt, op_t (&o)[NP]) {
#pragma unroll
                for (int p = 0; p < NP; ++p) o[p] = lds_operand<MODE>(Sg + bt * 8 * pitch + p * NCC * pitch + ks * KS);
              };
              static_for<0, 2>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                constexpr int m = GU::G.u[W][k][0], j0 = GU::G.u[W][k][1], j1 = GU::G.u[W][k][2];
                if constexpr (m >= 0) {
                  op_t a0[NP], a1[NP], bb[2][NP];
                  opnd(2 * m, a0);
                  if constexpr (2 * m + 1 < NCT) opnd(2 * m + 1, a1);
                  opnd(j0, bb[0]);
                  static_for<0, j1 - j0>([&](auto jc) {
                    constexpr int jj = decltype(jc)::value, j = j0 + jj;
                    if constexpr (jj + 1 < j1 - j0) opnd(j + 1, bb[(jj + 1) & 1]);
                    if (j < nbt) {                                          // uniform
                      static_for<0, 2>([&](auto rc) {
                        constexpr int r = decltype(rc)::value;
                        if constexpr (GU::tile_ok(2 * m + r, j)) {
                          constexpr int sl = GU::slot(W, k, jj, r);
                          if ((wkeep >> sl) & 1) {
                            accv_t acc = gacc[sl];
#pragma unroll
                            for (int pr = 0; pr < Traits<MODE>::NPROD; ++pr)
                              acc = mfma((r == 0 ? a0 : a1)[NP == 1 ? 0 : prod_a(NP, pr)],
                                         bb[jj & 1][NP == 1 ? 0 : prod_b(NP, pr)], acc);
                            gacc[sl] = acc;
                          }
                        }
                      });
                    }
                  });
                }
              });
            }
          }
        };
        switch (w) {
          case 0: run(std::integral_constant<int, 0>{}); break;
          case 1: run(std::integral_constant<int, 1>{}); break;
          case 2: run(std::integral_constant<int, 2>{}); break;
          case 3: run(std::integral_constant<int, 3>{}); break;
          case 4: run(std::integral_constant<int, 4>{}); break;
          case 5: run(std::integral_constant<int, 5>{}); break;
          case 6: run(std::integral_constant<int, 6>{}); break;
          default: run(std::integral_constant<int, 7>{}); break;
        }
        return;
      }
      if constexpr (NP == 3) {
        // six-product mode: one tile at a time (two tiles' operands in flight do not fit)
#pragma unroll
        for (int s = 0; s < C::NPW; ++s) {
          if (!((wkeep >> s) & 1)) continue;
          accv_t acc = gacc[s];
          for (int g = 0; g < ng; ++g) {
            const lds_t *SA, *SB;
            bases(s, g, SA, SB);
#pragma unroll 1
            for (int ks = 0; ks < KSN; ++ks) {
              op_t ao[NP], bo[NP];
              ld(SA, SB, ks, ao, bo);
#pragma unroll
              for (int pr = 0; pr < Traits<MODE>::NPROD; ++pr) acc = mfma(ao[prod_a(NP, pr)], bo[prod_b(NP, pr)], acc);
            }
          }
          gacc[s] = acc;
          __builtin_amdgcn_sched_barrier(0);
        }
        return;
      }
      for (int g = 0; g < ng; ++g) {
        op_t ao[2][NP], bo[2][NP];
        const lds_t *SA, *SB;
        bases(0, g, SA, SB);
        ld(SA, SB, 0, ao[0], bo[0]);
#pragma unroll
        for (int s = 0; s < C::NPW; ++s) {
          const bool valid = (wkeep >> s) & 1;                           // uniform
          const lds_t *nA = SA, *nB = SB;
          if (s + 1 < C::NPW) bases(s + 1, g, nA, nB);
          accv_t acc = gacc[s];
#pragma unroll 1
          for (int ks = 0; ks < KSN; ks += 2) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              if (ks + u + 1 < KSN) ld(SA, SB, ks + u + 1, ao[u ^ 1], bo[u ^ 1]);
              else if (s + 1 < C::NPW) ld(nA, nB, 0, ao[u ^ 1], bo[u ^ 1]);
              if (valid) {
#pragma unroll
                for (int pr = 0; pr < Traits<MODE>::NPROD; ++pr)
                  acc = mfma(ao[u][NP == 1 ? 0 : prod_a(NP, pr)], bo[u][NP == 1 ? 0 : prod_b(NP, pr)], acc);
              }
            }
          }
          gacc[s] = acc;
          SA = nA;
          SB = nB;
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    };

    for (int gbase = wi.g0; gbase < wi.g1; gbase += wi.ngc) {
      const int ng = min(wi.ngc, wi.g1 - gbase);
      const int ncols = ng * nb8;
      auto col_index = [&](int c, int& n) -> long {
        const int g = (int)__umulhi((uint32_t)c, nb8_rcp);
        n = c - g * nb8;
        return (long)(gbase + g) * nb + n;
      };

      // ================= multipole-free rows (block-sparse) =================
      // Per chunk of whole channels (at most GR rows and MPC multipole rows) the item's M values
      // of the chunk's rows are staged in LDS, XC columns at a time, and each lane takes one
      // column: a wavefront computes four rows of nearly equal run length at a time, each row r
      // of channel c as Y_s[r] = l_c[i] A[multipole row of c] + sum_{t < len} conj(L_c[i+t][i])
      // A[r + t] (the triangle without the padding to the chunk's longest run), its coefficients
      // read from the chunk's table by every lane at one address, A[r + t] from the stage (one
      // LDS read per term and column). The FP64 sums of |Y|^2 stay in registers, one per lane and column group. The
      // next stage's values come to registers while the current one runs; the workgroup meets
      // twice per stage (stage written, stage read) and once per chunk to contract its rows.
      if (a.n_s > 0 && wi.rb0 == 0) {
        constexpr int MAXT = C::MAXT, MPC = C::MPC, XC = C::XC, XP = C::XP, NU = C::NU;
        constexpr int NDR = C::NDR, XLD = C::XLD, XLM = C::XLM, LDRS = C::LDRS;
        const int nck = a.n_schunk;
        const int nstg = (ncols + XC - 1) / XC;
        double2* Cf = (double2*)(smem + C::SP_CF);            // [MAXT][GR] coefficient runs of the chunk
        int4* RI = (int4*)(smem + C::SP_RI);                   // [GR] {run start in coef, run length, multipole row}
        double2* CV = (double2*)(smem + C::SP_CV);             // [GR] l_c of each row
        uint2* GT = (uint2*)(smem + C::SP_GT);                 // [GR / 4] row groups of the chunk
        uint2* Xs = (uint2*)(smem + C::SP_X);                  // [GR + MPC][XP] complex64
        lds_t* Ss = (lds_t*)(smem + C::SP_ST);
        double dreg[NDR];
#pragma unroll
        for (int d = 0; d < NDR; ++d) dreg[d] = 0.0;
        auto chunk_info = [&](int ck) -> int4 {
          const int4 v = s_chunk[ck];
          return make_int4(uni(v.x), uni(v.y), uni(v.z), uni(v.w));
        };
        // the chunk's tables, one chunk ahead in registers: coefficients (all threads), row info
        // (threads 0 .. GR-1), l_c (threads GR .. 2 GR - 1) and row groups (the next GR / 4)
        constexpr int CFN = MAXT * GR;
        constexpr int CFL = (CFN + NT - 1) / NT;
        u4_t cfn[CFL];
        u4_t tabn;
        auto load_tab = [&](int ck) {
          const u4_t* src = (const u4_t*)(a.coefpad + pi.q * a.pad_qs + (long)ck * MAXT * GR);
#pragma unroll
          for (int i = 0; i < CFL; ++i)
            if (tid + NT * i < CFN) cfn[i] = src[tid + NT * i];
          const int4 ci = chunk_info(ck);
          tabn = u4_t{0u, 0u, 0u, 0u};
          if (tid < ci.y) {
            const int4 ri = a.rowinfo[ci.x + tid];
            tabn = u4_t{(uint32_t)ri.x, (uint32_t)ri.y, (uint32_t)(ri.z - ci.w), 0u};
          } else if (tid >= GR && tid - GR < ci.y) {
            tabn = __builtin_bit_cast(u4_t, a.cvec[pi.q * a.cvec_qs + ci.x + tid - GR]);
          } else if (tid >= 2 * GR && tid < 2 * GR + GR / 4) {
            const uint2 g = a.sgroup[(long)ck * (GR / 4) + tid - 2 * GR];
            tabn = u4_t{g.x, g.y, 0u, 0u};
          }
        };
        auto store_tab = [&]() {
#pragma unroll
          for (int i = 0; i < CFL; ++i)
            if (tid + NT * i < CFN) ((u4_t*)Cf)[tid + NT * i] = cfn[i];
          if (tid < GR) ((u4_t*)RI)[tid] = tabn;
          else if (tid < 2 * GR) ((u4_t*)CV)[tid - GR] = tabn;
          else if (tid < 2 * GR + GR / 4) GT[tid - 2 * GR] = make_uint2(tabn[0], tabn[1]);
        };
        // one stage's M values to registers: rows (lane = row, XLD columns per thread) and
        // multipole rows (16 lanes a column); columns past the item's read zero
        uint2 xr[XLD], xm[XLM];
        auto fetch = [&](int ck, int sg) {
          const int4 ci = chunk_info(ck);
          const int c0 = sg * XC;
#pragma unroll
          for (int j = 0; j < XLD; ++j) {
            const int cl = w + NW * j;                        // stage column
            const int c = c0 + cl;
            int n = 0;
            const long col = col_index(c, n);
            const bool ok = cl < XC && c < ncols && n < nb && lane < ci.y;
            xr[j] = buf_load<uint2>(mrs, ok ? (uint32_t)((col * pi.nmb + ci.x + lane) * esz) : 0x80000000u, 0u);
          }
#pragma unroll
          for (int j = 0; j < XLM; ++j) {
            const int e = (w + NW * j) * 64 + lane;
            const int cl = e / MPC, mr = e % MPC;
            const int c = c0 + cl;
            int n = 0;
            const long col = col_index(c, n);
            const bool ok = cl < XC && c < ncols && n < nb;
            xm[j] = buf_load<uint2>(mrs, ok ? (uint32_t)((col * pi.nmb + ci.w + mr) * esz) : 0x80000000u, 0u);
          }
        };
        auto put_stage = [&]() {
#pragma unroll
          for (int j = 0; j < XLD; ++j) {
            const int cl = w + NW * j;
            if (cl < XC) Xs[lane * XP + cl] = xr[j];
          }
#pragma unroll
          for (int j = 0; j < XLM; ++j) {
            const int e = (w + NW * j) * 64 + lane;
            const int cl = e / MPC, mr = e % MPC;
            if (cl < XC) Xs[(GR + mr) * XP + cl] = xm[j];
          }
        };
        auto to_d2 = [&](uint2 v) -> double2 {
          return make_double2((double)__uint_as_float(v.x), (double)__uint_as_float(v.y));
        };

        __syncthreads();                                      // earlier users of the LDS are done
        for (int e = tid; e < nck; e += NT) s_chunk[e] = a.schunk[e];
        __syncthreads();
        load_tab(0);
        store_tab();
        if (nck > 1) load_tab(1);
        fetch(0, 0);
        put_stage();
        __syncthreads();                                      // first stage and tables visible
        for (int ck = 0; ck < nck; ++ck) {
          for (int sg = 0; sg < nstg; ++sg) {
            // this lane's stage columns (a lane past the stage reads its last column, unused)
            int xo[NU];
#pragma unroll
            for (int u = 0; u < NU; ++u) xo[u] = min(u * 64 + lane, XC - 1);
            // the chunk's row groups (four rows of nearly equal run length each; rows past the
            // chunk have run length 0 and l_c = 0 and store the zeros the contraction reads),
            // dealt to the wavefronts in snake order; the four rows run together to their longest
            // run, the shorter ones on zero coefficients
            constexpr int NG = GR / 4;
            for (int rd = 0; rd * NW < NG; ++rd) {
              const uint2 gv = GT[rd * NW + ((rd & 1) ? NW - 1 - w : w)];
              const uint32_t packed = uni((int)gv.x);
              const int trip = uni((int)gv.y);
              int rr[4], len[4];
              double2 y[4][NU];
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                rr[e] = (packed >> (8 * e)) & 0xFF;
                const int4 ri = RI[rr[e]];
                len[e] = uni(ri.y);
                const int mloc = uni(ri.z);
                const double2 lc = CV[rr[e]];
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                  const double2 xm_ = to_d2(Xs[(GR + mloc) * XP + xo[u]]);
                  y[e][u].x = lc.x * xm_.x - lc.y * xm_.y;
                  y[e][u].y = lc.x * xm_.y + lc.y * xm_.x;
                }
              }
              auto term = [&](int e, const double2 l, int row) {
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                  const double2 x = to_d2(Xs[row * XP + xo[u]]);
                  y[e][u].x = fma(l.x, x.x, y[e][u].x);
                  y[e][u].y = fma(l.x, x.y, y[e][u].y);
                  y[e][u].x = fma(l.y, x.y, y[e][u].x);
                  y[e][u].y = fma(-l.y, x.x, y[e][u].y);
                }
              };
              // past a row's run its table entries are zero and its rows r + t < GR + MAXT stay in
              // the stage
              // per term: the four coefficients and 4 NU values requested together, then the FMAs
              const int tn = min(trip, MAXT);
              for (int t = 0; t < tn; ++t) {
                double2 lv[4];
                uint2 xv[4][NU];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  lv[e] = Cf[t * GR + rr[e]];
#pragma unroll
                  for (int u = 0; u < NU; ++u) xv[e][u] = Xs[(rr[e] + t) * XP + xo[u]];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                  for (int u = 0; u < NU; ++u) {
                    const double2 x = to_d2(xv[e][u]);
                    const double2 l = lv[e];
                    y[e][u].x = fma(l.x, x.x, y[e][u].x);
                    y[e][u].y = fma(l.x, x.y, y[e][u].y);
                    y[e][u].x = fma(l.y, x.y, y[e][u].x);
                    y[e][u].y = fma(-l.y, x.x, y[e][u].y);
                  }
              }
              for (int t = MAXT; t < trip; ++t) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                  const int cs = uni(RI[rr[e]].x);
                  term(e, t < len[e] ? a.coef[pi.q * a.coef_qs + cs + t] : make_double2(0.0, 0.0),
                       min(rr[e] + t, GR + MPC - 1));
                }
              }
#pragma unroll
              for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                  const int cl = u * 64 + lane, c = sg * XC + cl;
                  if (cl < XC && c < NCC) {
                    put_real<MODE>(Ss + (0 * NP) * NCC * LDRS + c * LDRS + rr[e], NCC * LDRS, y[e][u].x);
                    put_real<MODE>(Ss + (1 * NP) * NCC * LDRS + c * LDRS + rr[e], NCC * LDRS, y[e][u].y);
                    const double d = y[e][u].x * y[e][u].x + y[e][u].y * y[e][u].y;
#pragma unroll
                    for (int dd = 0; dd < NDR; ++dd)
                      if (dd == (sg * XC + u * 64) / 64) dreg[dd] += d;
                  }
                }
            }
            // the next stage's values are requested now and land during the barrier and the
            // contraction (they are not held in registers during the rows above)
            const bool more = sg + 1 < nstg || ck + 1 < nck;
            if (sg + 1 < nstg) fetch(ck, sg + 1);
            else if (ck + 1 < nck) fetch(ck + 1, 0);
            __syncthreads();                                  // the stage is read (and the chunk's rows staged)
            if (sg + 1 == nstg) {
              if (ck + 1 < nck) {
                store_tab();                                  // the next chunk's tables
                if (ck + 2 < nck) load_tab(ck + 2);
              }
              contract(Ss, ng, std::integral_constant<int, GR>{}, LDRS, std::true_type{});
            }
            if (more) put_stage();
            __syncthreads();                                  // next stage, tables visible; Gram stage free
          }
        }
#pragma unroll
        for (int dd = 0; dd < NDR; ++dd) {
          const int c = dd * 64 + lane;
          if (c < NCC) Dacc[(w * NCC + c) * 2] += dreg[dd];
        }
      }

      // ================= dense rows: row blocks of BM rows =================
      // the item's row parts: [rb0, rb1), part 0 the block-sparse rows, part 1 + j dense row block j
      const int r_lo = max(wi.rb0 - 1, 0) * BM, r_hi = min(nd, (wi.rb1 - 1) * BM);
      for (int r0 = r_lo; r0 < r_hi; r0 += BM) {
        accv_t acc[RT][NCT];
#pragma unroll
        for (int ii = 0; ii < RT; ++ii)
#pragma unroll
          for (int j = 0; j < NCT; ++j) acc[ii][j] = accv_t{0, 0, 0, 0};
        const int kc0 = (r0 / KC) * KC;
        const int kend = (nd + KC - 1) / KC * KC;
        const int np = (kend - kc0) / KC;                // K panels of this row block (>= 1)

        // direct loads of a raw panel: instruction t of this wavefront moves 1 KB = four columns
        // of KC complex64 values (16 lanes a column, two values a lane); instructions past the
        // panel's NI land in the trash KB, columns past the item's read zero
        uint32_t r_off[NIW];
        {
          int lane_d = lane;
          asm volatile("" : "+v"(lane_d));
#pragma unroll
          for (int t = 0; t < NIW; ++t) {
            const int ix = w + NW * t;
            const int c = ix * 4 + lane_d / 16;
            const int k = (lane_d % 16) * 2;
            int n = 0;
            const long col = col_index(c, n);
            const bool ok = ix < NI && c < ncols && n < nb;
            r_off[t] = ok ? (uint32_t)((col * pi.nmb + a.n_s + k) * esz) : 0x80000000u;
          }
        }
        auto issue_raw = [&](int kc, int buf) {
#pragma unroll
          for (int t = 0; t < NIW; ++t) {
            const int ix = w + NW * t;
            unsigned char* dst = ix < NI ? Raw + buf * C::RAW_B + ix * 1024 : Trash;
            lds_load16(mrs, dst, r_off[t], (uint32_t)(kc * esz));
          }
        };
        // raw panel -> pieces: thread u converts column u / (KC/8), k = 8 (u % (KC/8)) .. +7, four
        // k at a time; rows past N_d are zero
        auto convert_half = [&](int kc, int rbuf, int pbuf, int hf) {
          constexpr int KG = KC / 8;
          if (tid < NCC * KG) {
            const int c = tid / KG, kg = tid % KG;
            const float* src = (const float*)(Raw + rbuf * C::RAW_B + (c * KC + kg * 8) * 8);
            lds_t* dst = Pcs + pbuf * PCS + c * KCP + kg * 8;
            {
              const f4_t v0 = *(const f4_t*)(src + 8 * hf), v1 = *(const f4_t*)(src + 8 * hf + 4);
              const int k0 = kc + kg * 8 + 4 * hf;
              const bool o0 = k0 < nd, o1 = k0 + 1 < nd, o2 = k0 + 2 < nd, o3 = k0 + 3 < nd;
              store_pieces4<MODE>(dst + 4 * hf, APL, o0 ? v0[0] : 0.f, o1 ? v0[2] : 0.f, o2 ? v1[0] : 0.f,
                                  o3 ? v1[2] : 0.f);
              store_pieces4<MODE>(dst + NP * APL + 4 * hf, APL, o0 ? v0[1] : 0.f, o1 ? v0[3] : 0.f,
                                  o2 ? v1[1] : 0.f, o3 ? v1[3] : 0.f);
            }
          }
        };
        auto convert = [&](int kc, int rbuf, int pbuf) {
          convert_half(kc, rbuf, pbuf, 0);
          convert_half(kc, rbuf, pbuf, 1);
        };
        // factor pieces of this wave's two row tiles (w and w + NW of the block) for the panel at kc:
        // lane (l16, lq) holds row l16, k = 8 lq .. 8 lq + 7 of each piece plane (Re, then Im). The
        // matrix-core step ks takes k = 8 lq + ks from every lane group (bf16: one step over all 32
        // k; FP32: eight steps), the same permutation of k for both operands. Rows past N_d or
        // below the diagonal hold zeros (their products are skipped anyway).
        using ureg_t = typename std::conditional<MODE == M_F32, f4_t, u4_t>::type;
        constexpr int UPV = MODE == M_F32 ? 2 : NP;       // 16-byte registers per (row tile, Re/Im)
        ureg_t ucur[RT][2][UPV];
        // one half (h = 0: Re, 1: Im) of the factor pieces: NFL / 2 loads. The Re half of the
        // next panel is requested in the middle of the current one, once its last product with
        // the Re half has been issued, the Im half at its end: each half has half a panel of
        // products to land in.
        // A tile that starts at or past N_d reads zeros: its rows may lie past the factor's
        // padded order, and only the per-lane offset is checked against the buffer's size.
        auto load_u_h = [&](int kc, int h) {
#pragma unroll
          for (int ii = 0; ii < RT; ++ii) {
            const int tr = r0 + 16 * (w + NW * ii);
            const bool live = tr < nd;                    // uniform
            const long row0 = (long)tr * pi.ldu + kc;
#pragma unroll
            for (int v = 0; v < UPV; ++v) {
              const long e = MODE == M_F32 ? h * plane + row0 + 4 * v : (h * NP + v) * plane + row0;
              ucur[ii][h][v] = buf_load<ureg_t>(urs, live ? u_lane : 0x80000000u, live ? (uint32_t)(e * C::ESZ) : 0u);
            }
          }
        };
        auto load_u = [&](int kc) {
          load_u_h(kc, 0);
          load_u_h(kc, 1);
        };
        // A operand of step ks, piece pa, from the registers above
        auto uop = [&](int ii, int h, int ks, int pa) -> op_t {
          if constexpr (MODE == M_F32) {
            return ucur[ii][h][ks >> 2][ks & 3];
          } else {
            (void)ks;
            return ucur[ii][h][pa];
          }
        };
        auto n_active = [&](int kc) {
          int n = 0;
#pragma unroll
          for (int ii = 0; ii < RT; ++ii)
            if (r0 + 16 * (w + NW * ii) < min(kc + KC, nd)) n = ii + 1;
          return n;
        };

        __syncthreads();                                  // LDS of the previous phase is free
        // prologue: raw panels 0 .. NRAW-1 in flight, then the factor of panel 0
        issue_raw(kc0, 0);
        if (np > 1) issue_raw(kc0 + KC, 1);
        if (NRAW == 3 && np > 2) issue_raw(kc0 + 2 * KC, 2);
        load_u(kc0);
        // own part of raw panel 0 landed: the later NIW (panels 1, 2) + NFL (factor) loads may fly
        if (NRAW == 3 && np > 2) wait_vm<2 * NIW + NFL>();
        else if (np > 1) wait_vm<NIW + NFL>();
        else wait_vm<NFL>();
        __syncthreads();
        convert(kc0, 0, 0);
        if (np > 1) {                                     // own part of raw panel 1 landed
          if (NRAW == 3 && np > 2) wait_vm<NIW + NFL>();
          else wait_vm<NFL>();
        }
        __syncthreads();

        for (int p = 0; p < np; ++p) {
          const int kc = kc0 + p * KC;
          // A: raw panel p + NRAW into the buffer panel p came in (converted before the last barrier)
          const bool issued = p + NRAW < np;
          if (issued) issue_raw(kc + NRAW * KC, p % NRAW);
          // B: the Re half of this panel's factor landed (its Im half and the raw loads just
          // issued may still fly)
          if (issued) wait_vm<NIW + NFL / 2>();
          else wait_vm<NFL / 2>();
          // the middle of the panel: the Im half landed (only the raw loads issued above may
          // still fly), then the Re half of the next panel's factor into the registers the
          // products with the Re half no longer read
          auto mid = [&]() {
            if (issued) wait_vm<NIW>();
            else wait_vm<0>();
            if (p + 1 < np) load_u_h(kc + KC, 0);
          };
          // C: [Yr|Yi] += Ur [Ar|Ai] + Ui [-Ai|Ar] over the panel
          const int na = n_active(kc);
          // per-panel lane addresses from an opaque lane copy (see contract): the B operand of
          // step (h, j) is plane part (h = 0) or, for h = 1, -Im (part 0) or Re (part 1), read at
          // column j 8 + c8 and k = 8 lq + ks (see load_u); every other term is an immediate offset
          int lx = lane;
          asm volatile("" : "+v"(lx));
          const int xpart = (lx >> 3) & 1;
          const lds_t* Pl = Pcs + (p & 1) * PCS + (lx & 7) * KCP + 8 * (lx >> 4);
          const lds_t* B0 = Pl + xpart * NP * APL;
          const lds_t* B1 = Pl + (1 - xpart) * NP * APL;
          // -Im for the real-part lanes of the h = 1 operand: a sign-bit mask, no branch
          const uint32_t nmask = xpart == 0 ? (MODE == M_F32 ? 0x80000000u : 0x80008000u) : 0u;
          // the panel's products for NA active row tiles (NA known at compile time: the loop
          // below is straight-line code with no per-instruction branches)
          // the next panel's conversion (VALU and LDS work of its own) goes between the
          // products, in two halves, so that it runs while the matrix cores work
          const bool conv = p + 1 < np;
          auto panel = [&](auto na_c) {
            constexpr int NA = decltype(na_c)::value;
#pragma unroll
            for (int ks = 0; ks < KC / KS; ++ks) {
              auto bload = [&](int hj, op_t (&b)[NP]) {
                const int h = hj / NCT, j = hj % NCT;
                const lds_t* Bh = h == 0 ? B0 : B1;
#pragma unroll
                for (int p2 = 0; p2 < NP; ++p2) {
                  b[p2] = lds_operand<MODE>(Bh + p2 * APL + j * 8 * KCP + ks);
                  if (h == 1) b[p2] = sign_flip(b[p2], nmask);
                }
              };
              op_t bA[NP], bB[NP];
              bload(0, bA);
#pragma unroll
              for (int hj = 0; hj < 2 * NCT; ++hj) {
                const int h = hj / NCT, j = hj % NCT;
                op_t (&bc)[NP] = (hj & 1) ? bB : bA;
                op_t (&bn)[NP] = (hj & 1) ? bA : bB;
                if (hj + 1 < 2 * NCT) bload(hj + 1, bn);
#pragma unroll
                for (int pr = 0; pr < Traits<MODE>::NPROD; ++pr)
#pragma unroll
                  for (int ii = 0; ii < NA; ++ii)
                    acc[ii][j] = mfma(uop(ii, h, ks, NP == 1 ? 0 : prod_a(NP, pr)),
                                      bc[NP == 1 ? 0 : prod_b(NP, pr)], acc[ii][j]);
                // keep the scheduler from hoisting later operand loads (register pressure)
                __builtin_amdgcn_sched_barrier(0);
                if (ks == KC / KS - 1 && (hj == NCT / 2 || hj == NCT + NCT / 2) && conv) {
                  convert_half(kc + KC, (p + 1) % NRAW, (p + 1) & 1, hj == NCT / 2 ? 0 : 1);
                  __builtin_amdgcn_sched_barrier(0);
                }
                if (ks == KC / KS - 1 && hj == NCT - 1) {
                  mid();
                  __builtin_amdgcn_sched_barrier(0);
                }
              }
            }
          };
          if (na > 0) {
            panel(std::integral_constant<int, RT>{});
          } else {
            mid();
            if (conv) convert(kc + KC, (p + 1) % NRAW, (p + 1) & 1);
          }
          if (p + 1 < np) {
            // (E, the next panel's pieces from its raw panel -- landed and visible since the
            // last barrier -- into the other piece buffer, ran between the products above)
            // D: the Im half of the next panel's factor, after the products that read this one's
            load_u_h(kc + KC, 1);
            // F: own part of raw panel p + 2 landed, for the conversion after the next barrier.
            // Loads issued after it: NRAW = 3 -> both halves of this panel's factor (the middle
            // and the end of the last panel), raw p + 3 (A above, if issued) and both halves of
            // the next panel's; NRAW = 2 -> both halves of the next panel's factor.
            if (p + 2 < np) {
              if constexpr (NRAW == 3) {
                if (issued) wait_vm<NIW + 2 * NFL>();
                else wait_vm<2 * NFL>();
              } else {
                wait_vm<NFL>();
              }
            }
          }
          __syncthreads();
        }

        // ---- the row block's rows through LDS into the Gram tiles, GS rows at a time ----
        constexpr int RPS = GS / 16;                      // row tiles per stage round
#pragma unroll
        for (int rr = 0; rr < BM / GS; ++rr) {
          if (r0 + rr * GS >= nd) break;                  // uniform
          __syncthreads();                                // the stage is free
          // lane addresses from an opaque lane copy (see contract): column c8 of the part's
          // plane, rows 4 lq .. 4 lq + 3 of the tile (the accumulator rows of the lane)
          int lx = lane;
          asm volatile("" : "+v"(lx));
          const int xlq = lx >> 4, xpart = (lx >> 3) & 1;
          lds_t* Yl = Ys + (xpart * NP) * NCC * LDR + (lx & 7) * LDR + 4 * xlq;
          double* Dl = Dacc + (w * NCC + (lx & 7)) * 2 + xpart;
#pragma unroll
          for (int ii = 0; ii < RT; ++ii) {
            const int tile = w + NW * ii;                 // this wave's row tile in the block
            if (tile / RPS != rr) continue;
            const int trow = (tile % RPS) * 16;
            const int rlim = nd - (r0 + rr * GS + trow + 4 * xlq);   // rows of the lane below N_d
#pragma unroll
            for (int j = 0; j < NCT; ++j) {
              double d = 0.0;
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const float y = e < rlim ? (float)acc[ii][j][e] : 0.f;
                put_realf<MODE>(Yl + j * 8 * LDR + trow + e, NCC * LDR, y);
                d += (double)y * (double)y;
              }
              d += __shfl_xor(d, 16);
              d += __shfl_xor(d, 32);
              if (xlq == 0) Dl[j * 16] += d;
            }
          }
          __syncthreads();
          contract(Ys, ng, std::integral_constant<int, GS>{}, LDR, std::true_type{});
        }
      }
      // ---- this n'' chunk's Gram tiles into the item's partial slot (stored by the first
      // chunk, added by the others): each chunk's sums over the mixed basis run in their own
      // binary32 accumulators, as one (pair, n'') slot would hold them, and the chunks of an
      // item meet in one binary32 addition each instead of one sequential sum over every row
      // of every n''
#pragma unroll
      for (int s = 0; s < C::NPW; ++s) {
        const int tp = slot_tp(s);
        if (tp >= 0 && tp < npt) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc_t* d = gp + (tp * 4 + i) * 64 + lane;
            *d = gbase == wi.g0 ? gacc[s][i] : *d + gacc[s][i];
          }
        }
        gacc[s] = accv_t{0, 0, 0, 0};
      }
    }  // n'' chunks

    __syncthreads();
    for (int n = tid; n < nb8; n += NT) {
      double s = 0.0;
      for (int c = n; c < NCC; c += nb8)
        for (int ww = 0; ww < NW; ++ww) s += Dacc[(ww * NCC + c) * 2] + Dacc[(ww * NCC + c) * 2 + 1];
      a.dpart[(long)wi.slot * a.dstride + n] = s;
    }
    if (tid0 == 0) s_item = claim;
    __syncthreads();
    idx = -1;
    if (home) {
      const int j = qh0 + n_static(qi) + __builtin_amdgcn_readfirstlane(s_item);
      if (j < qh1) idx = j;
      else home = false;
    }
    __syncthreads();
  }
}

}  // namespace exc
