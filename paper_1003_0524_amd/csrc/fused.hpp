// Fused exchange kernel for the reduced-precision Cholesky/HERK form: one work
// item (pair (k,q), a range of n'' values) reads its columns of M once and
// produces the item's Gram partial
//
//   G = sum_{n''} Y_{n''}^H Y_{n''},   Y = [ Y_s ; Y_d ],
//   Y_s = L_c^H A_c + l_c a_{j(c)}   (block-sparse multipole-free rows, FP64 VALU)
//   Y_d = L22^H A_d                  (dense rows, MFMA in the mode's pieces)
//
// the vector-matrix-vector form of Sec. III.C with v = L L^H and the sparse
// structure of the transformed Coulomb matrix (Fig. 1).
//
// Layout of the work in one workgroup (4 wavefronts, one per SIMD):
//  * multipole-free rows, in chunks of whole channels of at most GR = 64 rows
//    (lane = row): each wavefront forms Y_s of its own columns in FP64 registers
//    (the rows a coefficient run needs come from the lanes below by DPP shifts),
//    writes the split pieces to LDS and keeps |Y|^2 for the FP64 diagonal in
//    registers; then the Gram tiles are contracted over the chunk on MFMA;
//  * dense rows, in row blocks of BM = 64 RTW rows: the accumulators of the
//    whole row block live in registers (wavefront w owns row tiles w, w+4, ...);
//    the K loop starts at the block's first row (L22^H is upper triangular),
//    streams raw K panels of A_d global -> LDS (two in flight where LDS allows),
//    converts each into the mode's pieces of Re, Im and -Im, and reads the
//    factor's pieces straight from global memory (L2: the factor of q is shared
//    by every k); then the rows go through LDS, GR at a time, into the Gram
//    contraction.
// Partials: one slot per item (Gram tiles in accumulator order and the FP64
// diagonal per band), summed per k in a fixed order by the reduction kernel.
#pragma once
#include "common.hpp"
#include "tile.hpp"

#include <type_traits>

namespace exc {

// Lane l takes the value of lane l + 1 (the last lane takes zero): a whole-wavefront DPP
// shift, per 32-bit half.
__device__ __forceinline__ double shift_down1(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x130, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double2 shift_down1(double2 v) { return make_double2(shift_down1(v.x), shift_down1(v.y)); }

// Work queues of the persistent launch: NQ queues (one per XCD: consecutive
// workgroups are dispatched to the 8 XCDs in turn, so workgroup b serves queue
// b % NQ first), each a range of the item array. The first item of every workgroup
// is fixed (workgroup b takes item b / NQ of its queue); the rest are claimed with
// the queue's atomic counter, one item ahead (the claim is issued when an item
// starts and read when it ends: counters shared by the XCDs are far away). A
// workgroup whose queue is empty reads all counters at once and takes items from
// queues that still have some.
constexpr int NQ_MAX = 8;

struct FusedArgs {
  const PairInfo* pairs;
  const WorkItem* items;
  int32_t n_items;
  int32_t* counter;               // non-null: persistent mode ([nq] counters)
  const int32_t* qbeg;            // [nq + 1] item range of each queue (persistent mode)
  int32_t nq;
  const void* const* mtab;
  int32_t m_c64;
  int32_t n_s, n_ch, n_occ;
  const void* U;                  // prepared factor planes
  const int32_t* row_chan;
  const int32_t* ch_off;
  const int32_t* ch_len;
  const int64_t* ch_coef;
  const double2* coef;            // L_c (column-major, per channel)
  const double2* cvec;            // l_c per multipole-free row
  const int4* schunk;             // chunks of whole channels, at most 64 rows and 16 multipole rows:
  int32_t n_schunk;               //  {first row, rows, longest run, first multipole row}
  const double2* coefpad;         // per chunk, [MAXT][64]: the first MAXT entries of each row's
                                  // run (transposed), zero padded
  int64_t coef_qs, cvec_qs, pad_qs;   // elements between the copies of q and q + 1 of coef,
                                      // cvec and coefpad (0: one copy for all q)
  const int4* rowinfo;            // per multipole-free row r of channel c (r = first row + i):
                                  // {index in coef of conj-coefficient run L_c[i..b-1][i], b - i,
                                  //  multipole row n_s + c, 0}
  const uint2* sgroup;            // per chunk, 16 groups of four of its 64 rows (rows past the chunk
                                  // with run length 0) by decreasing run length: {rows (one byte
                                  // each), longest run}
  void* gpart;
  double* dpart;
  int32_t gstride, dstride;
  const uint64_t* tmask;          // [n_k][3] band-tile pairs to compute (bit tp), nullptr: all
};

template <int MODE, int RTW, int NCT, int NB8M, int KC, int CBX = 16, int OCC = 1>
struct FusedCfg {
  using T = Traits<MODE>;
  using lds_t = typename T::lds_t;
  using acc_t = typename T::acc_t;
  using accv_t = typename T::accv_t;
  static constexpr int NW = 4, NT = 256;
  static constexpr int NRT = 4 * RTW, BM = 16 * NRT;   // row tiles / rows of a dense row block
  static constexpr int GR = 64;                         // rows per Gram chunk (one row tile per wavefront)
  static constexpr int NP = T::NPIECE, KS = T::KS, KPL = KS / 4, NPL = 2 * NP;
  static constexpr int NCC = NCT * 8;
  static constexpr int ESZ = (int)sizeof(lds_t);
  static constexpr int EPV = 16 / ESZ;                  // elements per 16 bytes
  static constexpr int LDK = KC + EPV;                  // A panel pitch (k contiguous per column)
  static constexpr int APL = NCC * LDK;
  // converted panel: pieces of Re, Im and, where it fits the LDS share, -Im (else the
  // MFMA loop negates Im)
  static constexpr bool NEGP = (size_t)(3 * NP * NCC * LDK * ESZ) + (NCC * KC * 16 + 4095) / 4096 * 4096 +
                                   (size_t)NW * NCC * 2 * sizeof(double) + 16 * 64 + 32 <= (size_t)163840 / OCC;
  static constexpr int ABUF = (NEGP ? 3 : 2) * NP * APL;
  static constexpr int LDR = GR + EPV;                  // Gram stage pitch (rows contiguous per column)
  static constexpr int YPL = NCC * LDR;
  static constexpr int YS = NPL * YPL;
  static constexpr int NPT = NB8M * (NB8M + 1) / 2;
  static constexpr int NPW = (NPT + NW - 1) / NW;
  static constexpr bool GSTREAM = NPW > 8;
  // binary32 Gram chains (for error models): one per item, or (GSTREAM) one per GR-row
  // chunk added into the item's partial; GR rows per chunk in both row kinds
  static constexpr int GCHAIN = GSTREAM ? 1 : 0, GCH_RS = GR, GCH_RD = GR;
  static constexpr int CB = CBX;                         // sparse step: columns (CB / NW per wavefront)
  static constexpr int CPW = CB / NW;
  static constexpr int NCB = (NCC + CB - 1) / CB;        // column blocks of a sparse chunk (at most)
  static constexpr int MAXT = 12;                        // coefficients per row staged in LDS (longer runs: global)
  static constexpr int CFL = MAXT * GR / NT;             // coefficient table: 16-byte loads per thread
  static constexpr int MPC = GR / CPW;                   // multipole rows per sparse chunk (at most)
  static constexpr int MAXCK = 64;                       // sparse chunks (at most)
  static constexpr int SP_MP = 0;                        // sparse phase LDS: [NW][CPW][MPC] multipole rows,
  static constexpr int SP_CF = SP_MP + CB * MPC * 16;    // [MAXT][GR] coefficients,
  static constexpr int SP_ST = SP_CF + MAXT * GR * 16;   // then the Gram stage
  static constexpr int SPARSE_B = SP_ST + YS * ESZ;
  static constexpr int RAW_B = (NCC * KC * 16 + 4095) / 4096 * 4096;   // raw panel (complex128 worst case), a whole
                                                                       // number of 1 KB loads per wavefront
  static constexpr int PL_B = ABUF * ESZ;               // converted panel
  // two raw panel buffers where they fit the LDS share (with the other phases' needs)
  static constexpr size_t FIXED_B = (size_t)NW * NCC * 2 * sizeof(double) + 16 * MAXCK + 16;
  static constexpr size_t MAXSHARE = 163840 / OCC;
  static constexpr size_t OTHER_B = (size_t)(SPARSE_B > YS * ESZ ? SPARSE_B : YS * ESZ);
  static constexpr int NRAW = (2 * (size_t)RAW_B + PL_B <= MAXSHARE - FIXED_B - 16) ? 2 : 1;
  static constexpr size_t DENSE_B = (size_t)(NRAW * RAW_B + PL_B > OTHER_B ? NRAW * RAW_B + PL_B : OTHER_B);
  static constexpr size_t MAIN_RAW = DENSE_B > (size_t)SPARSE_B ? DENSE_B : (size_t)SPARSE_B;
  static constexpr size_t MAIN_B = (MAIN_RAW + 15) / 16 * 16;
  // s_waitcnt immediate for vmcnt(0) alone (gfx9 encoding: expcnt and lgkmcnt at their maxima)
  static constexpr int WAIT_VM0 = 0x0F70;
  // vmcnt(NIW): all but the last NIW vector-memory instructions of the wavefront
  static constexpr int NIW_C = RAW_B / 1024 / NW;
  static constexpr int WAIT_VM_NIW = (NIW_C & 0xF) | ((NIW_C >> 4) << 14) | 0x0F70;
  static_assert(NIW_C < 64, "vmcnt is a 6-bit count");
  static constexpr size_t DACC_B = (size_t)NW * NCC * 2 * sizeof(double);
  static constexpr size_t LDS_B = MAIN_B + DACC_B;
  static_assert(MODE != M_F64, "the fused kernel serves the reduced-precision modes");
  static_assert(RTW >= 1 && RTW <= 5, "one to five row tiles per wavefront");
  static_assert(KC % KS == 0 && KC % EPV == 0, "K panel is a whole number of MFMA steps");
  static_assert(GR % KS == 0, "Gram chunk is a whole number of MFMA steps");
  static_assert(LDS_B + 16 * MAXCK + 16 <= 163840 / OCC, "fused configuration exceeds its share of the 160 KB of LDS");
  static_assert(CB % NW == 0 && CB >= NW, "sparse step: whole columns per wavefront");
  static_assert((MAXT * GR) % NT == 0, "coefficient table: whole loads per thread");
  static_assert(CPW * MPC == 64, "one multipole block load per wavefront and sparse step");
};

// REALF: the factor and the channel couplings are real (inversion symmetry): the
// products with their imaginary parts, which are zero, are left out.
template <int MODE, int RTW, int NCT, int NB8M, int KC, int CBX = 16, int OCC = 1, bool REALF = false>
__global__ __launch_bounds__(256, OCC) void fused_kernel(FusedArgs a) {
  using C = FusedCfg<MODE, RTW, NCT, NB8M, KC, CBX, OCC>;
  using lds_t = typename C::lds_t;
  using acc_t = typename C::acc_t;
  using accv_t = typename C::accv_t;
  using op_t = decltype(lds_operand<MODE>((const lds_t*)nullptr));
  constexpr int NW = C::NW, NT = C::NT, NP = C::NP, KS = C::KS, KPL = C::KPL, NPL = C::NPL;
  constexpr int NCC = C::NCC, LDK = C::LDK, APL = C::APL, LDR = C::LDR, YPL = C::YPL, GR = C::GR;
  constexpr int EPV = C::EPV, BM = C::BM, NRT = C::NRT;

  __shared__ __align__(16) unsigned char smem[C::LDS_B];
  __shared__ int s_item;
  __shared__ int4 s_chunk[C::MAXCK];
  unsigned char* Raw = smem;                   // NRAW x [NCC][KC] complex, as loaded (K loop)
  lds_t* Apl = (lds_t*)(smem + C::NRAW * C::RAW_B);   // [3 NP][NCC][LDK] pieces (K loop)
  lds_t* Ys = (lds_t*)smem;                    // [NPL][NCC][LDR] (Gram stage; aliases the K panels)
  double* Dacc = (double*)(smem + C::MAIN_B);  // [NW][NCC][2]

  const int tid0 = threadIdx.x;

  __shared__ int s_left[NQ_MAX];
  const int nq = a.counter ? a.nq : 1;
  const int G = (int)gridDim.x;
  const int qi = a.counter ? (int)(blockIdx.x % nq) : 0;
  auto n_static = [&](int q) { return (G - q + nq - 1) / nq; };   // workgroups whose first queue is q
  int qh0 = 0, qh1 = 0;                           // the first queue's item range
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
  // an item of another queue, or -1 when every queue is drained
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
    int claim = 0;                                // the first queue's next item, claimed now
    if (home && tid0 == 0) claim = atomicAdd(a.counter + qi, 1);

    // Lane indices, derived afresh for every item from a copy of the thread index that the
    // compiler cannot see through: values computed from them (addresses, masks) are not
    // hoisted out of the item loop and kept live, in registers or spilled, for the whole
    // kernel.
    int tid_o = tid0;
    asm volatile("" : "+v"(tid_o));
    const int tid = tid_o, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: branches on it stay scalar
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
    const int esz = a.m_c64 ? 8 : 16;
    const char* mbase = uni((const char*)a.mtab[pi.k]) + pi.m_off * esz;
    const __amdgpu_buffer_rsrc_t mrs = make_rsrc(mbase, (uint32_t)((long)a.n_occ * nb * pi.nmb * esz));
    const lds_t* Ug = (const lds_t*)a.U + pi.u_off;
    const long plane = (long)pi.ldu * pi.ldu;
    const __amdgpu_buffer_rsrc_t urs = make_rsrc(Ug, (uint32_t)(NPL * plane * C::ESZ));
    const uint32_t u_lane = (uint32_t)((l16 * pi.ldu + KPL * lq) * C::ESZ);

    constexpr int NPWR = C::GSTREAM ? 1 : C::NPW;
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
    for (int e = tid; e < NW * NCC * 2; e += NT) Dacc[e] = 0.0;
    // this wavefront's tiles (bit s: tile w + NW s) that the band mask of k keeps
    const uint64_t wkeep = tile_keep_bits(a.tmask, pi.k, w, NW, C::NPW);

    // ---- contraction of the staged GR rows into this wave's Gram tiles ----
    // rows_c: rows of the stage (GR), pitch: its row pitch
    auto contract_chunk = [&](const lds_t* Ys, int ng, auto rows_c, int pitch) {
      constexpr int ROWS = decltype(rows_c)::value;
      auto one = [&](int tp, accv_t acc) -> accv_t {
        int I, J;
        tp_to_ij(tp, I, J);
        for (int g = 0; g < ng; ++g) {
          const int cA = g * nb8 + I * 8 + c8, cB = g * nb8 + J * 8 + c8;
#pragma unroll
          for (int ks = 0; ks < ROWS / KS; ++ks) {
            const int kofs = ks * KS + KPL * lq;
            op_t ao[NP], bo[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
              ao[p] = lds_operand<MODE>(Ys + (part * NP + p) * NCC * pitch + cA * pitch + kofs);
              bo[p] = lds_operand<MODE>(Ys + (part * NP + p) * NCC * pitch + cB * pitch + kofs);
            }
            if constexpr (NP == 1) {
              acc = mfma(ao[0], bo[0], acc);
            } else {
#pragma unroll
              for (int pr = 0; pr < C::T::NPROD; ++pr) acc = mfma(ao[prod_a(NP, pr)], bo[prod_b(NP, pr)], acc);
            }
          }
        }
        return acc;
      };
      if constexpr (C::GSTREAM) {
        for (int s = 0; s < C::NPW; ++s) {
          const int tp = w + NW * s;
          if (tp >= npt) break;
          if (!((wkeep >> s) & 1)) continue;
          const accv_t acc = one(tp, accv_t{0, 0, 0, 0});
#pragma unroll
          for (int i = 0; i < 4; ++i) gp[(tp * 4 + i) * 64 + lane] += acc[i];
        }
      } else {
#pragma unroll
        for (int s = 0; s < NPWR; ++s) {
          const int tp = w + NW * s;
          if (tp < npt && ((wkeep >> s) & 1)) gacc[s] = one(tp, gacc[s]);
        }
      }
    };

    for (int gbase = wi.g0; gbase < wi.g1; gbase += wi.ngc) {
      const int ng = min(wi.ngc, wi.g1 - gbase);
      const int ncols = ng * nb8;
      // item column -> M column (n'', n); n >= nb: padding. c / nb8 as a multiply-high by
      // ceil(2^32 / nb8), exact for c * nb8 < 2^32
      auto col_index = [&](int c, int& n) -> long {
        const int g = (int)__umulhi((uint32_t)c, nb8_rcp);
        n = c - g * nb8;
        return (long)(gbase + g) * nb + n;
      };

      // ================= multipole-free rows (block-sparse) =================
      // Chunks of whole channels of at most GR rows (lane = row of the chunk) whose
      // multipole rows lie within MPC consecutive rows, so that every run L_c[i..b-1][i]
      // meets rows of its own chunk only. A step is one chunk and a block of CB columns;
      // wavefront w owns the columns w, w + NW, ... of the block: their rows of M (one
      // per lane) and the chunk's multipole rows (one 16-row block per column) come to
      // registers two steps ahead (two register sets, used in turn). Y_s is computed in
      // registers: term t of a row's run needs the row t below it, which the lane gets
      // by shifting the column's values down one lane per term (DPP), so each term costs
      // one LDS read (its coefficient, shared by the lane's CPW columns) and no barrier.
      // The workgroup meets once per chunk, when every column is staged, to contract it.
      // The FP64 sums of |Y|^2 stay in registers, one per lane (row) and column, and are
      // summed over the rows once at the end.
      if (a.n_s > 0 && wi.rb0 == 0) {
        constexpr int CB = C::CB, CPW = C::CPW, NCB = C::NCB, MAXT = C::MAXT, CFL = C::CFL, MPC = C::MPC;
        const int nck = a.n_schunk;
        const int ncb = (ncols + CB - 1) / CB;
        const int nsteps = nck * ncb;
        double2* Mp = (double2*)(smem + C::SP_MP + w * CPW * MPC * 16);   // this wavefront's [CPW][MPC] multipole rows
        double2* Cf = (double2*)(smem + C::SP_CF);            // [MAXT][GR] coefficient runs of the chunk
        lds_t* Ss = (lds_t*)(smem + C::SP_ST);                // [NPL][NCC][LDR] Gram stage
        double dreg[NCB][CPW];
#pragma unroll
        for (int b = 0; b < NCB; ++b)
#pragma unroll
          for (int j = 0; j < CPW; ++j) dreg[b][j] = 0.0;

        struct RowData { double2 lc; int cs, len, mloc; };
        auto chunk_info = [&](int ck) -> int4 {       // {first row, rows, longest run, first multipole row}
          const int4 v = s_chunk[ck];
          return make_int4(uni(v.x), uni(v.y), uni(v.z), uni(v.w));
        };
        auto load_rows = [&](const int4& ci, RowData& d) {
          d.len = 0; d.cs = 0; d.mloc = 0;
          d.lc = make_double2(0.0, 0.0);
          if (lane < ci.y) {
            const int4 ri = a.rowinfo[ci.x + lane];
            d.cs = ri.x; d.len = ri.y; d.mloc = ri.z - ci.w;
            d.lc = a.cvec[pi.q * a.cvec_qs + ci.x + lane];
          }
        };
        u4_t cfn[CFL];                                // the next chunk's coefficient table
        auto load_coef = [&](int ck) {
          const u4_t* src = (const u4_t*)(a.coefpad + pi.q * a.pad_qs + (long)ck * MAXT * GR);
#pragma unroll
          for (int i = 0; i < CFL; ++i) cfn[i] = src[tid + NT * i];
        };
        auto store_coef = [&]() {
#pragma unroll
          for (int i = 0; i < CFL; ++i) ((u4_t*)Cf)[tid + NT * i] = cfn[i];
        };
        // one step's values of M: xn[j] = row (first + lane) of column j, pn = multipole
        // row (first multipole row + lane % MPC) of column lane / MPC
        struct StepRegs { u4_t xn[CPW]; u4_t pn; };
        auto fetch = [&](int st, StepRegs& X) {
          const int4 ci = chunk_info(st / ncb);
          const int cb0 = (st % ncb) * CB;
#pragma unroll
          for (int j = 0; j < CPW; ++j) {
            const int c = cb0 + w + NW * j;
            int n = 0;
            const long col = col_index(c, n);
            const bool ok = c < ncols && n < nb && lane < ci.y;
            const uint32_t vx = ok ? (uint32_t)((col * pi.nmb + ci.x + lane) * esz) : 0x80000000u;
            if (a.m_c64) {
              const uint2 x = buf_load<uint2>(mrs, vx, 0u);
              X.xn[j] = u4_t{x.x, x.y, 0u, 0u};
            } else {
              X.xn[j] = buf_load<u4_t>(mrs, vx, 0u);
            }
          }
          {
            const int c = cb0 + w + NW * (lane / MPC);
            int n = 0;
            const long col = col_index(c, n);
            const bool ok = c < ncols && n < nb;
            const uint32_t vm = ok ? (uint32_t)((col * pi.nmb + ci.w + lane % MPC) * esz) : 0x80000000u;
            if (a.m_c64) {
              const uint2 m = buf_load<uint2>(mrs, vm, 0u);
              X.pn = u4_t{m.x, m.y, 0u, 0u};
            } else {
              X.pn = buf_load<u4_t>(mrs, vm, 0u);
            }
          }
        };
        auto to_d2 = [&](u4_t v) -> double2 {
          if (a.m_c64) return make_double2((double)__uint_as_float(v.x), (double)__uint_as_float(v.y));
          return make_double2(__hiloint2double((int)v.y, (int)v.x), __hiloint2double((int)v.w, (int)v.z));
        };

        __syncthreads();                              // earlier users of the LDS are done
        for (int e = tid; e < nck; e += NT) s_chunk[e] = a.schunk[e];
        load_coef(0);
        store_coef();
        __syncthreads();                              // chunk table and first coefficients visible
        int4 ci = chunk_info(0);
        RowData rd, rd_next;
        load_rows(ci, rd);
        rd_next = rd;
        if (nck > 1) {
          load_rows(chunk_info(1), rd_next);
          load_coef(1);
        }
        StepRegs SA, SB;
        fetch(0, SA);
        if (nsteps > 1) fetch(1, SB);

        auto step = [&](int st, StepRegs& X) {
          const int cbk = st % ncb, cb0 = cbk * CB;
          // this step's values to registers (rows) and to the wavefront's LDS slots
          // (multipole rows), then the step two ahead into X
          double2 xs[CPW];
#pragma unroll
          for (int j = 0; j < CPW; ++j) xs[j] = to_d2(X.xn[j]);
          Mp[lane] = to_d2(X.pn);
          if (st + 2 < nsteps) fetch(st + 2, X);
          // LDS operations of one wavefront take effect in order: the slots just written
          // are read below by other lanes of the same wavefront
          __builtin_amdgcn_wave_barrier();
          // Y_s[r] = sum_{j >= i} conj(L_c[j][i]) A[first + j] + l_c[i] A[multipole row of c]
          double2 y[CPW];
#pragma unroll
          for (int j = 0; j < CPW; ++j) {
            const double2 xm = Mp[j * MPC + rd.mloc];
            if constexpr (REALF) {
              y[j].x = rd.lc.x * xm.x;
              y[j].y = rd.lc.x * xm.y;
            } else {
              y[j].x = rd.lc.x * xm.x - rd.lc.y * xm.y;
              y[j].y = rd.lc.x * xm.y + rd.lc.y * xm.x;
            }
          }
          // Term t: coefficient L_c[i+t][i] (zero past the row's run, in the table) times
          // the value of row r + t, which xs holds after t shifts (zero past the chunk:
          // lanes past the chunk hold zeros and the last lane takes in zero). All lanes
          // run the chunk's longest run and shift together.
          auto term = [&](const double2 l) {
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
              y[j].x = fma(l.x, xs[j].x, y[j].x);
              y[j].y = fma(l.x, xs[j].y, y[j].y);
              if constexpr (!REALF) {
                y[j].x = fma(l.y, xs[j].y, y[j].x);
                y[j].y = fma(-l.y, xs[j].x, y[j].y);
              }
              xs[j] = shift_down1(xs[j]);
            }
          };
          const int T = min(ci.z, MAXT);
          for (int t = 0; t < T; ++t) term(Cf[t * GR + lane]);
          for (int t = MAXT; t < ci.z; ++t)           // runs longer than the staged table
            term(t < rd.len ? a.coef[pi.q * a.coef_qs + rd.cs + t] : make_double2(0.0, 0.0));
#pragma unroll
          for (int j = 0; j < CPW; ++j) {
            const int c = cb0 + w + NW * j;
            if (c < NCC) {
              put_real<MODE>(Ss + (0 * NP) * NCC * LDR + c * LDR + lane, NCC * LDR, y[j].x);
              put_real<MODE>(Ss + (1 * NP) * NCC * LDR + c * LDR + lane, NCC * LDR, y[j].y);
            }
            const double d = y[j].x * y[j].x + y[j].y * y[j].y;
#pragma unroll
            for (int b = 0; b < NCB; ++b)
              if (b == cbk) dreg[b][j] += d;
          }
          if (cbk == ncb - 1) {                       // the chunk's columns are staged
            __syncthreads();                          // (its coefficients are no longer read)
            const int ck = st / ncb;
            if (ck + 1 < nck) {
              store_coef();
              ci = chunk_info(ck + 1);
              rd = rd_next;
              if (ck + 2 < nck) {
                load_rows(chunk_info(ck + 2), rd_next);
                load_coef(ck + 2);
              }
            }
            contract_chunk(Ss, ng, std::integral_constant<int, GR>{}, LDR);
            __syncthreads();                          // the stage is free, the next coefficients visible
          }
        };
        for (int st = 0; st < nsteps; st += 2) {
          step(st, SA);
          if (st + 1 < nsteps) step(st + 1, SB);
        }
#pragma unroll
        for (int b = 0; b < NCB; ++b)
#pragma unroll
          for (int j = 0; j < CPW; ++j) {
            double d = dreg[b][j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
            const int c = b * CB + w + NW * j;
            if (lane == 0 && c < NCC) Dacc[(w * NCC + c) * 2] += d;
          }
      }

      // ================= dense rows: row blocks of BM rows =================
      // the item's row parts: [rb0, rb1), part 0 the block-sparse rows, part 1 + j dense row block j
      const int r_lo = max(wi.rb0 - 1, 0) * BM, r_hi = min(nd, (wi.rb1 - 1) * BM);
      for (int r0 = r_lo; r0 < r_hi; r0 += BM) {
        accv_t acc[RTW][NCT];
#pragma unroll
        for (int ii = 0; ii < RTW; ++ii)
#pragma unroll
          for (int j = 0; j < NCT; ++j) acc[ii][j] = accv_t{0, 0, 0, 0};
        const int kc0 = (r0 / KC) * KC;
        const int kend = (nd + KC - 1) / KC * KC;
        const int nrt_nd = (nd - r0 + 15) / 16;          // row tiles holding rows < nd

        // ---- K panels of A_d: global -> LDS directly (buffer_load ... lds), then
        // converted in LDS into the mode's pieces. One wave instruction moves 1 KB:
        // two columns of KC complex128 (or four of complex64), lanes in order. With
        // NRAW = 2 raw buffers two panels are in flight; the factor pieces of a panel are
        // requested before its raw panel two ahead, so that waiting for them (vmcnt counts
        // in order) leaves that panel in flight; every wavefront issues the same NIW raw
        // instructions per panel (past the data's end they read zero).
        constexpr int NI = C::RAW_B / 1024;                // instructions per panel
        constexpr int NIW = (NI + NW - 1) / NW;            // per wavefront
        uint32_t r_off[NIW];
        {
          const int cpi = a.m_c64 ? 4 : 2;                 // columns per instruction
          const int lpc = 64 / cpi;                        // lanes per column
          int lane_d = lane;                               // (not hoisted above the sparse phase)
          asm volatile("" : "+v"(lane_d));
#pragma unroll
          for (int t = 0; t < NIW; ++t) {
            const int idx = w + NW * t;
            const int c = idx * cpi + lane_d / lpc;
            const int k = (lane_d % lpc) * (a.m_c64 ? 2 : 1);
            int n = 0;
            const long col = col_index(c, n);
            const bool ok = idx < NI && c < ncols && n < nb && c * KC * esz < C::RAW_B;
            // invalid columns: an offset past the end of any pair block (2 GiB; no wrap-around
            // with the scalar offset added) reads zero
            r_off[t] = ok ? (uint32_t)((col * pi.nmb + a.n_s + k) * esz) : 0x80000000u;
          }
        }
        auto issue_raw = [&](int kc, int buf) {
#pragma unroll
          for (int t = 0; t < NIW; ++t)
            lds_load16(mrs, Raw + buf * C::RAW_B + (w + NW * t) * 1024, r_off[t], (uint32_t)(kc * esz));
        };
        // raw -> pieces: consecutive lanes take consecutive elements (a wavefront reads
        // 1 KB of contiguous LDS per instruction, free of bank conflicts) and write
        // their pieces as single elements of the planes
        auto convert = [&](int kc, int buf) {
          const unsigned char* Rw = Raw + buf * C::RAW_B;
          for (int e = tid; e < NCC * KC; e += NT) {
            const int c = e / KC, k = e % KC;
            double re = 0.0, im = 0.0;
            if (kc + k < nd) {
              if (a.m_c64) {
                const float2 v = *(const float2*)(Rw + e * 8);
                re = (double)v.x;
                im = (double)v.y;
              } else {
                const double2 v = *(const double2*)(Rw + e * 16);
                re = v.x;
                im = v.y;
              }
            }
            if constexpr (C::NEGP && !REALF) {      // (a real factor never reads the -Im plane)
              put_cplx3<MODE>(Apl + c * LDK + k, APL, re, im);
            } else {
              put_real<MODE>(Apl + c * LDK + k, APL, re);
              put_real<MODE>(Apl + NP * APL + c * LDK + k, APL, im);
            }
          }
        };

        __syncthreads();                              // the stage is free
        // factor pieces of this wave's tiles for the current K panel, requested before the
        // panel's conversion (L2 latency hides behind it and the barrier that follows)
        op_t ucur[RTW][KC / KS][2][NP];
        // row tiles of this wavefront with a nonzero factor block in the K panel at kc:
        // L22^H is upper triangular, so tiles whose rows start past the panel's last k
        // (or past N_d) meet zeros only; the active tiles are a prefix in ii
        auto n_active = [&](int kc) {
          int n = 0;
#pragma unroll
          for (int ii = 0; ii < RTW; ++ii)
            if (r0 + 16 * (w + 4 * ii) < min(kc + KC, nd)) n = ii + 1;
          return n;
        };
        // tiles past the panel's triangle (or past N_d) read zeros through an out-of-range
        // per-lane offset: the products below run over every tile with no branch, and theirs add
        // exact zeros
        auto load_u = [&](int kc, op_t (&u)[RTW][KC / KS][2][NP]) {
          const int na = n_active(kc);
#pragma unroll
          for (int ii = 0; ii < RTW; ++ii) {
            const bool act = ii < na;                     // uniform
            const long row0 = (long)(r0 + 16 * (w + 4 * ii)) * pi.ldu + kc;
#pragma unroll
            for (int ks = 0; ks < KC / KS; ++ks)
#pragma unroll
              for (int h = 0; h < (REALF ? 1 : 2); ++h)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                  u[ii][ks][h][p] = buf_load<op_t>(
                      urs, act ? u_lane : 0x80000000u,
                      act ? (uint32_t)(((h * NP + p) * plane + row0 + ks * KS) * C::ESZ) : 0u);
          }
        };
        const int np = (kend - kc0) / KC;                 // K panels of this row block
        issue_raw(kc0, 0);
        if (C::NRAW == 2 && np > 1) {
          issue_raw(kc0 + KC, 1);
          __builtin_amdgcn_s_waitcnt(C::WAIT_VM_NIW);     // panel 0 has landed
        } else {
          __builtin_amdgcn_s_waitcnt(C::WAIT_VM0);
        }
        __syncthreads();
        for (int pp = 0; pp < np; ++pp) {
          const int kc = kc0 + pp * KC, buf = C::NRAW == 2 ? (pp & 1) : 0;
          load_u(kc, ucur);                           // this panel's factor pieces in flight
          convert(kc, buf);
          __syncthreads();                            // pieces ready, raw buffer free
          const bool more = pp + 1 < np;
          if (C::NRAW == 2) {
            if (pp + 2 < np) issue_raw(kc + 2 * KC, buf);
          } else if (more) {
            issue_raw(kc + KC, 0);
          }
          const int na = n_active(kc);                // uniform
          // -Im of the h = 1 operand where no -Im plane is staged: a sign-bit mask, no branch
          const uint32_t nmask = part == 0 ? (MODE == M_F32 ? 0x80000000u : 0x80008000u) : 0u;
          // [Yr|Yi] += Br [Ar|Ai] + Bi [-Ai|Ar]: the B operand of step (h, j) is plane
          // part (h = 0) or, for h = 1, -Im (part 0) or Re (part 1); one step ahead
#pragma unroll
          for (int ks = 0; ks < KC / KS; ++ks) {
            const int kofs = ks * KS + KPL * lq;
            auto bload = [&](int hj, op_t (&b)[NP]) {
              const int h = hj / NCT, j = hj % NCT;
              const int pl = C::NEGP ? (h == 0 ? part : 2 * (1 - part)) : (part ^ h);
#pragma unroll
              for (int p = 0; p < NP; ++p) {
                b[p] = lds_operand<MODE>(Apl + (pl * NP + p) * APL + (j * 8 + c8) * LDK + kofs);
                if (!C::NEGP && h == 1) b[p] = sign_flip(b[p], nmask);
              }
            };
            op_t bA[NP], bB[NP];
            bload(0, bA);
            constexpr int NHJ = (REALF ? 1 : 2) * NCT;      // a real factor has no Bi products
#pragma unroll
            for (int hj = 0; hj < NHJ; ++hj) {
              const int h = hj / NCT, j = hj % NCT;
              op_t (&bc)[NP] = (hj & 1) ? bB : bA;
              op_t (&bn)[NP] = (hj & 1) ? bA : bB;
              if (hj + 1 < NHJ) bload(hj + 1, bn);
              // products outer, tiles inner: consecutive MFMAs use different accumulators
#pragma unroll
              for (int pr = 0; pr < C::T::NPROD; ++pr)
#pragma unroll
                for (int ii = 0; ii < RTW; ++ii)
                  if (MODE != M_F32 || ii < na)   // (fp32: its cheaper products of zero tiles still cost more)
                    acc[ii][j] = mfma(ucur[ii][ks][h][NP == 1 ? 0 : prod_a(NP, pr)],
                                      bc[NP == 1 ? 0 : prod_b(NP, pr)], acc[ii][j]);
            }
          }
          // this wave's part of the next panel has landed
          if (C::NRAW == 2 && pp + 2 < np) __builtin_amdgcn_s_waitcnt(C::WAIT_VM_NIW);
          else __builtin_amdgcn_s_waitcnt(C::WAIT_VM0);
          __syncthreads();
        }

        // ---- the row block's rows through LDS into the Gram tiles, GR rows at a time ----
#pragma unroll
        for (int ii = 0; ii < RTW; ++ii) {
          if (r0 + ii * GR >= nd) break;              // uniform
          __syncthreads();                            // the stage is free
#pragma unroll
          for (int j = 0; j < NCT; ++j) {
            const int cl = j * 8 + c8;
            double d = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int row = w * 16 + acc_row<MODE>(lq, e);
              // rows past N_d: the factor rows read there belong to padding or other planes
              const float y = (r0 + ii * GR + row < nd) ? (float)acc[ii][j][e] : 0.f;
              put_realf<MODE>(Ys + (part * NP) * YPL + cl * LDR + row, YPL, y);
              d += (double)y * (double)y;
            }
            d += __shfl_xor(d, 16);
            d += __shfl_xor(d, 32);
            if (lq == 0) Dacc[(w * NCC + cl) * 2 + part] += d;
          }
          __syncthreads();
          contract_chunk(Ys, ng, std::integral_constant<int, GR>{}, LDR);
        }
      }
    }  // n'' chunks

    // ---- the item's partials ----
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
    __syncthreads();                              // s_item is read before the next item writes it
  }
}

}  // namespace exc
