// jz_stage_kernel.h -- fused residual + Runge-Kutta stage kernel, templated
// over the arithmetic type (FP64 path and FP32-flux path).
//
// One launch performs one stage Q(k) = Q(0) - alpha_k dt R(Q(k-1)) over the
// whole block (Sec. 3: explicit multistage scheme; Sec. 4.2: each stage runs
// the full residual -- inviscid flux, viscosity update, viscous flux and
// artificial dissipation).  R = J (C - D):
//   C = sum_d delta_d Fhat^d, Fhat^d = sum_a S^d_a (E_a - V_a)       (Eqs. (vec-les), (con-prop))
//   E_a inviscid flux; V_a viscous flux from the Stokes stress (Eq. (tau_mod)),
//   Sutherland (Eq. (sutherland)) plus Smagorinsky viscosity and the heat
//   flux of Eq. (q_mod); gradients are nodal centred differences mapped with
//   the metrics, so the viscous part reaches two nodes out;
//   D = sum_d (d_{i+1/2} - d_{i-1/2}), the scalar anisotropic dissipation
//   with second/fourth differences on the five-point stencil (Sec. 4.3).
//
// Work decomposition (2.5-D march):
//   * a workgroup covers an in-plane tile of TI x TJ owned columns plus a
//     two-node halo ring, and marches along zeta over a chunk of planes;
//   * each thread owns one (i, j) column of the tile and keeps the
//     zeta-direction neighbours of its column in registers (three planes of
//     Q, the zeta flux and dissipation terms it needs next);
//   * threads are assigned by role so that whole wavefronts skip the work
//     their nodes do not need: owned columns first (they do everything), then
//     the first halo ring without its corners (they need fluxes for one
//     direction), then the nodes that only supply primitives and Q (ring-1
//     corners, ring-2 edges); ring-2 corners are never read and get no thread;
//   * in-plane neighbours are exchanged through LDS, one plane at a time:
//     primitives, Q and p of the gradient plane; then the xi/eta fluxes,
//     dissipation scales and pressure sensors of the same plane;
//   * per march step s the lead plane s+2 is loaded, the gradient plane s+1
//     gets its fluxes, and plane s gets its residual and is written.
// Along a periodic direction every global access uses wrapped indices, so
// the halo is the block's own periodic image (standing in for the
// neighbour-rank ghost layers of Sec. 4.3).  Along a direction with physical
// faces the tiles cover only the interior nodes; the two boundary layers at
// each end are read as halo (the boundary conditions set them after every
// stage) and never written here.  Inside the library Q is stored node-major (the five
// conserved variables of a node contiguous, 40 B) and the metric set likewise
// (10 doubles, 80 B per node): one address per node and array, and a
// wavefront still reads one contiguous span per plane row.
//
// Precision forms (template parameters Rl, TIn, TOut, MET32):
//   FP64:      everything in double; metrics node-major, 10 doubles per node.
//   FP32-flux: primitives, gradients, viscosities, fluxes and dissipation in
//              float, read from a float copy of the stencil input (stages 2-5)
//              and float metrics (9 per node); J stays double, R = J (C - D)
//              is formed in double and Q(k) = Q(0) - alpha_k dt R is
//              accumulated in double from the double Q(0); intermediate stage
//              states are stored in float (they only feed the next stage's
//              stencil), the last stage stores double.  Residual norms and the
//              CFL reduction stay double.
#pragma once

#include <stdint.h>
#include <type_traits>
#include "jz_internal.h"

namespace jz {

namespace {

template <typename Rl>
struct Prim {
  Rl u, v, w, T, p;
};

template <typename Rl>
__device__ inline Prim<Rl> primitives(const Rl q[5], Rl gm1, Rl gamma) {
  Prim<Rl> r;
  const Rl rinv = rcp_pos(q[0]);
  r.u = q[1] * rinv;
  r.v = q[2] * rinv;
  r.w = q[3] * rinv;
  r.p = gm1 * (q[4] - Rl(0.5) * q[0] * (r.u * r.u + r.v * r.v + r.w * r.w));
  r.T = gamma * r.p * rinv;
  return r;
}

// J^(-1/3) (the filter width of a cell of volume 1/J): float seed from the
// hardware log2/exp2, then two Newton steps r <- r + r (1 - J r^3) / 3 in FP64,
// which square the relative error twice (1e-7 -> 1e-14 -> below rounding).
__device__ inline double inv_cbrt(double J) {
  const float jf = (float)J;
  double r = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(jf) * (1.0f / 3.0f));
  r = r + r * (1.0 - J * r * r * r) * (1.0 / 3.0);
  r = r + r * (1.0 - J * r * r * r) * (1.0 / 3.0);
  return r;
}

// J^(-1/3) in float: hardware log2/exp2 seed and one Newton step
__device__ inline float inv_cbrt(float J) {
  float r = __builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(J) * (1.0f / 3.0f));
  return r + r * (1.0f - J * r * r * r) * (1.0f / 3.0f);
}

// A register copy the compiler cannot fold into its source: the result gets
// registers of its own (early clobber), distinct from the operand's.
__device__ inline double move_apart(double x) {
  double y;
  asm volatile("v_mov_b64 %0, %1" : "=&v"(y) : "v"(x));
  return y;
}
__device__ inline float move_apart(float x) {
  float y;
  asm volatile("v_mov_b32 %0, %1" : "=&v"(y) : "v"(x));
  return y;
}



// Role of thread t in a TI x TJ tile with a two-node halo: position (tx, ty)
// in the (TI+4) x (TJ+4) tile and role 0 = owned column, 1 = first-ring edge
// (needs fluxes), 2 = primitives and Q only, 3 = idle.
template <int TI, int TJ>
__device__ inline int tile_role(int t, int& tx, int& ty) {
  constexpr int NI = TI * TJ, NR = 2 * TI + 2 * TJ;
  if (t < NI) {
    tx = 2 + t % TI;
    ty = 2 + t / TI;
    return 0;
  }
  int r = t - NI;
  int ring = 1, role = 1;
  if (r >= NR) {
    r -= NR;
    role = 2;
    if (r < 4) {  // first-ring corners
      tx = (r & 1) ? TI + 2 : 1;
      ty = (r & 2) ? TJ + 2 : 1;
      return 2;
    }
    r -= 4;
    if (r >= NR) {
      tx = ty = 0;
      return 3;
    }
    ring = 2;
  }
  const int lo = 2 - ring, hi_i = TI + 1 + ring, hi_j = TJ + 1 + ring;
  if (r < TI) {
    tx = 2 + r;
    ty = lo;
  } else if (r < 2 * TI) {
    tx = 2 + r - TI;
    ty = hi_j;
  } else if (r < 2 * TI + TJ) {
    tx = lo;
    ty = 2 + r - 2 * TI;
  } else {
    tx = hi_i;
    ty = 2 + r - 2 * TI - TJ;
  }
  return role;
}

// Role of thread t in the compact form: t < TI TJ owns a column; the next
// 2 TI + 2 TJ threads are the first-ring edge nodes (role 1, in the order of
// tile_role) and also carry the second-ring node (tx2, ty2) outward of their
// edge; the next four the first-ring corners (role 2); the rest are idle.
template <int TI, int TJ>
__device__ inline int tile_role_compact(int t, int& tx, int& ty, int& tx2, int& ty2) {
  constexpr int NI = TI * TJ;
  tx2 = ty2 = 0;
  if (t < NI) {
    tx = 2 + t % TI;
    ty = 2 + t / TI;
    return 0;
  }
  int r = t - NI;
  if (r < 2 * TI) {
    tx = tx2 = 2 + r % TI;
    ty = r < TI ? 1 : TJ + 2;
    ty2 = r < TI ? 0 : TJ + 3;
    return 1;
  }
  r -= 2 * TI;
  if (r < 2 * TJ) {
    ty = ty2 = 2 + r % TJ;
    tx = r < TJ ? 1 : TI + 2;
    tx2 = r < TJ ? 0 : TI + 3;
    return 1;
  }
  r -= 2 * TJ;
  if (r < 4) {
    tx = (r & 1) ? TI + 2 : 1;
    ty = (r & 2) ? TJ + 2 : 1;
    return 2;
  }
  tx = ty = 0;
  return 3;
}

// Owned-phase helpers.  In the FP64 shapes with 256 owned columns (four
// waves, one per SIMD) the workgroup has 512 threads, and thread NI + l is the
// partner of owned thread l: the same SIMD, otherwise busy only with the
// halo's primitives and fluxes.  In the owned phase the partner computes the
// in-plane terms of the last three conserved variables of the owner's column,
// so that two waves per SIMD share that phase (the owner keeps two, the zeta
// face and the update).
template <typename Rl, int BX, int BY>
constexpr bool stage_helpers() { return sizeof(Rl) == 8 && (BX - 4) * (BY - 4) == 256; }
// Compact form (FP64 tiles of 16 x 12 owned columns): 256 threads, one wave
// per SIMD.  The 192 owned columns and the 56 first-ring edge nodes fill the
// four waves, so every SIMD runs exactly one flux stream per plane; each edge
// thread also supplies the second-ring node outward of its edge (primitives
// and Q only), and four threads the first-ring corners.  At two waves per
// SIMD a CU holds two such workgroups, whose barriers and latencies then
// overlap with the other's work.
template <typename Rl, int BX, int BY>
constexpr bool stage_compact() { return sizeof(Rl) == 8 && BX == 20 && BY == 16; }
template <typename Rl, int BX, int BY>
constexpr int stage_threads() {
  return stage_compact<Rl, BX, BY>() ? 256 : stage_helpers<Rl, BX, BY>() ? 512 : BX * BY;
}
// conserved variables whose in-plane terms the partner computes
template <typename Rl, int BX, int BY>
constexpr int stage_helper_vars() { return stage_helpers<Rl, BX, BY>() ? 3 : 0; }

// Row pitch (in slots) of the LDS plane buffers of a BX x BY workgroup.  With
// a pitch of BX, the slots of one tile column lie BX elements apart and the
// halo threads that walk a column hit the same LDS bank on every row; one
// slot of padding per row spreads them over the banks.  The padding is taken
// where the plane buffers of a stage with the primitive ring (39, plus the
// partners' terms for two march steps; slots up to the last one a thread
// uses: ring-2 corners have none; 32 bytes of alignment slack) still let the
// CU hold the workgroups the register budget allows: two waves per SIMD in
// FP64, three in the FP32-flux form.
template <typename Rl, int BX, int BY>
constexpr long long lds_plane_bytes(int pitch) {
  return (39LL + 2 * stage_helper_vars<Rl, BX, BY>()) * ((BX - 2) + (long long)pitch * (BY - 1)) *
             (long long)sizeof(Rl) + 32;
}
template <typename Rl, int BX, int BY>
constexpr int lds_pitch() {
  constexpr long long kLds = 160 * 1024;
  constexpr int waves = sizeof(Rl) == 4 ? 3 : 2;
  constexpr int nth = stage_threads<Rl, BX, BY>();
  constexpr long long want = (waves * 4 * 64 + nth - 1) / nth;  // workgroups for that many waves
  constexpr long long fit = kLds / lds_plane_bytes<Rl, BX, BY>(BX);
  return kLds / lds_plane_bytes<Rl, BX, BY>(BX + 1) >= (want < fit ? want : fit) ? BX + 1 : BX;
}

}  // namespace

// MODE bit 0: accumulate norms of R (first stage)
// MODE bit 1: max of sum_d lambda^d of the updated state (last stage -> next dt)
// MODE bit 2: write R itself instead of the stage update
// MODE bit 3: a float stage state of a block with far-field faces: keep the
//             double update of the reference planes (StageArgs::ref)
// One tile (logical index lt of the block described by A) through one stage.
// Partial norms and lambda maxima go to slot lt, so the reductions do not
// depend on how tiles are scheduled.  Every thread of the workgroup calls it;
// PERSIST: called from the persistent batch kernel's tile loop.
template <typename Rl, typename TIn, typename TOut, bool MET32, int BX, int BY, int MODE, bool PERSIST>
__device__ __forceinline__ void stage_tile(const StageArgs& A, const int lt) {
  constexpr int NT = stage_threads<Rl, BX, BY>();  // threads of the workgroup
  constexpr int TI = BX - 4, TJ = BY - 4;
  constexpr int NI = TI * TJ;                       // owned columns
  constexpr bool HELP = stage_helpers<Rl, BX, BY>();
  constexpr int NHV = stage_helper_vars<Rl, BX, BY>();  // variables its helper computes
  constexpr int NV_OWN = 5 - NHV;                   // variables the owner's owned phase computes
  constexpr int P = lds_pitch<Rl, BX, BY>();   // LDS row pitch
  constexpr int NS = (BX - 2) + P * (BY - 1);   // LDS slots per plane buffer
  constexpr bool NORMS = (MODE & 1) != 0;
  constexpr bool LAMMAX = (MODE & 2) != 0;
  constexpr bool WRITE_R = (MODE & 4) != 0;
  constexpr bool KEEP_REF = (MODE & 8) != 0 && std::is_same<TOut, float>::value && !PERSIST;
  constexpr int BASE = MODE & 7;  // the stage kind without bit 3
  constexpr bool COMPACT = stage_compact<Rl, BX, BY>();
  static_assert(COMPACT ? NI + 2 * TI + 2 * TJ + 4 <= NT : TI * TJ + 4 * TI + 4 * TJ + 4 <= NT,
                "tile roles exceed the workgroup");

  // The column's own primitives of planes s, s+1 and s+2 (the zeta
  // neighbours and the centre of the gradient plane) are kept in registers:
  // one plane of primitives in LDS instead of a ring of three, and 15 fewer
  // LDS reads per flux column.  Where the registers do not allow it, the
  // stage keeps the ring: the FP32-flux first stage (norms at three waves
  // per SIMD) and, in the batch kernel, whose tile loop holds more
  // registers, every stage with reductions -- except in the compact FP64
  // form, whose ring (93 KB of LDS) would leave one workgroup per CU: there
  // the registers spill 40-48 bytes per lane instead, which costs less.
  constexpr bool ZREG = BASE == 0 || ((!PERSIST || stage_compact<Rl, BX, BY>()) &&
                                      (BASE == 2 || (BASE == 1 && sizeof(Rl) == 8)));
  constexpr int NPR = ZREG ? 1 : 3;
  // plane buffers (structure of arrays, one slot per tile column, rows of P)
  __shared__ Rl sPr[NPR][5][NS];   // u, v, w, T, p: the gradient plane, or a ring of three planes
  // Q of the gradient plane, read in the owned phase after the second
  // barrier.  The compact form, whose LDS must hold two workgroups, keeps one
  // buffer and writes it after the first barrier of a march step (by then
  // every thread has finished reading the previous plane's Q); the other
  // shapes write before that barrier, alternating between two buffers.
  constexpr int NQB = COMPACT ? 1 : 2;
  __shared__ Rl sQ2[NQB][5][NS];
  __shared__ __attribute__((aligned(16))) Rl sF[10][NS];  // Fhat^xi (rows 0-4), Fhat^eta (rows 5-9)
  Rl(*sFx)[NS] = sF;
  Rl(*sFy)[NS] = sF + 5;
  __shared__ Rl sSx[NS], sSy[NS];  // sigma^xi, sigma^eta
  __shared__ Rl sNx[NS], sNy[NS];  // pressure sensor along xi, eta
  // helpers' in-plane terms of variables NV_OWN..4 of the owned columns, by march-step parity
  __shared__ Rl sRg[HELP ? 2 : 1][HELP ? NHV : 1][HELP ? NS : 1];
  // Last stage (single block): each owned thread keeps the metrics of its
  // column's gradient plane, which it has in registers for the fluxes, in
  // its own LDS slots (by plane parity) for the next-dt spectral radius of
  // that plane's update one march step later, instead of reading them from
  // memory again; no other thread touches them.  Only where the CU's LDS
  // holds them beside the plane buffers (29 with the primitives in
  // registers, and the partners' terms) for as many workgroups as the
  // registers allow (two waves per SIMD in FP64, three in the FP32-flux form).
  typedef typename std::conditional<MET32, float, double>::type MT;  // stored metric type
  constexpr long long MET_LDS_WG =
      (19LL + 5 * NQB + 2 * NHV) * NS * (long long)sizeof(Rl) + 2LL * NI * (9 * (long long)sizeof(MT) + 8) + 256;
  constexpr long long REG_WAVES = (sizeof(Rl) == 4 ? 3 : 2) * 4 * 64;
  constexpr long long REG_WG = REG_WAVES / NT > 0 ? REG_WAVES / NT : 1;
  constexpr bool MET_LDS = BASE == 2 && ZREG && !PERSIST && MET_LDS_WG * REG_WG <= 160LL * 1024;
  __shared__ MT sMo[MET_LDS ? 2 : 1][MET_LDS ? 9 : 1][MET_LDS ? NI : 1];
  __shared__ double sMoJ[MET_LDS ? 2 : 1][MET_LDS ? NI : 1];
  // Compact form: Q of the next gradient plane of each edge thread's
  // second-ring column goes straight from memory into LDS, without registers
  // (kept in registers, its loads would share them with the owned columns'
  // values, and the compiler, which cannot tell lanes apart, would then wait
  // for every load in flight at each march step).  Lane l of the edge wave
  // loads 4-byte word d of its node into sQB[d][l].  The loads are issued in
  // inline assembly right after the metric prefetch of the gradient phase:
  // the compiler does not see them, and none of its own loads issued before
  // that point is waited for until the next march step, by which time these
  // have landed; their reader waits for them explicitly (s_waitcnt vmcnt(0))
  // at the top of the next march step, before anything newer is issued.
  __shared__ uint32_t sQB[COMPACT ? 10 : 1][COMPACT ? 64 : 1];
  // end-of-tile reductions reuse the flux buffer (free once the march is done)
  static_assert(sizeof(Rl) * 10 * NS >= sizeof(double) * 2 * NT, "reduction rows exceed the flux buffer");
  double(*sRed)[NT] = reinterpret_cast<double(*)[NT]>(&sF[0][0]);

  const Phys ph = A.ph;
  const Rl gm1 = (Rl)ph.gm1, gamma = (Rl)ph.gamma;
  const Rl k2 = (Rl)ph.k2, k4 = (Rl)ph.k4;
  // Logical tile order: chunk by chunk, bands of RB tile rows cut into
  // segments of SW tiles along xi, and within a segment the band's rows
  // alternate along xi.  The workgroups that run at once on one XCD
  // (consecutive logical tiles) then form a compact patch, whose inner halo
  // rows and columns are read once into the L2.  The 512 workgroups of 16 x 12
  // tiles that run at once (64 per XCD) take patches of 8 x 8 tiles (0.7 %
  // faster than 4 x 16 and than 2 rows across the block); the other shapes
  // take bands of 2 rows across the block (about 5 % fewer HBM reads than one
  // tile row per XCD).  A last band or segment may be smaller.
  constexpr int RB = COMPACT ? 8 : 2;
  const int SW = COMPACT ? min(8, A.tiles_i) : A.tiles_i;
  const int per_chunk = A.tiles_i * A.tiles_j;
  const int chunk = lt / per_chunk;
  const int r = lt - chunk * per_chunk;
  const int band = r / (RB * A.tiles_i);
  const int rows = min(RB, A.tiles_j - RB * band);
  const int w = r - band * RB * A.tiles_i;
  const int seg = w / (rows * SW);
  const int v = w - seg * rows * SW;
  const int tile_i = seg * SW + v / rows;
  const int tile_j = RB * band + v % rows;
  const int i0 = A.in.lo[0] + tile_i * TI, j0 = A.in.lo[1] + tile_j * TJ;
  const int kbeg = A.in.lo[2] + chunk * A.kchunk;
  const int kend = min(kbeg + A.kchunk, A.in.hi[2]);

  const int t = threadIdx.x;
  int tx, ty, tx2 = 0, ty2 = 0;
  const int role = COMPACT ? tile_role_compact<TI, TJ>(t, tx, ty, tx2, ty2) : tile_role<TI, TJ>(t, tx, ty);
  const int c = tx + P * ty;                      // LDS slot of this column
  const int ui = i0 - 2 + tx, uj = j0 - 2 + ty;  // unwrapped column indices
  const bool bi = A.in.bnd & 1, bj = A.in.bnd & 2, bk = A.in.bnd & 4;
  const long long col = (long long)map_index(ui, A.ni, bi) + (long long)A.ni * map_index(uj, A.nj, bj);
  const long long plane = (long long)A.ni * A.nj;
  // compact form: the second-ring column an edge thread supplies (slot cB)
  const bool hasB = COMPACT && role == 1;
  const int cB = tx2 + P * ty2;
  const long long colB = COMPACT ? (long long)map_index(i0 - 2 + tx2, A.ni, bi) +
                                       (long long)A.ni * map_index(j0 - 2 + ty2, A.nj, bj)
                                 : 0;
  // supplies primitives and Q.  In the compact form the four idle threads
  // do too, for the never-read second-ring corner slot (0, 0): then every
  // lane issues the same prefetch loads (see below).
  const bool isP = role <= 2 || COMPACT;
  const bool isG = role <= 1;                     // computes fluxes
  const bool isI = role == 0 && ui < A.in.hi[0] && uj < A.in.hi[1];  // owns (writes) its column
  // the owned column this thread helps with (HELP: thread NI + l helps owned thread l)
  const int hl = t - NI;
  const int ch = HELP ? (2 + hl % TI) + P * (2 + hl / TI) : 0;
  const bool isH = HELP && t >= NI && t < 2 * NI && (i0 + hl % TI) < A.in.hi[0] && (j0 + hl / TI) < A.in.hi[1];

  const TIn* __restrict__ qin = (const TIn*)A.qin;
  TOut* __restrict__ qout = (TOut*)A.qout;
  MetView<MET32> met;
  met.m = (decltype(met.m))A.met;
  met.jac = A.jac;
  const double dt = A.clock->dt;
  const double adt = A.alpha * dt;
  const bool q0_is_input = (const void*)A.qin == (const void*)A.q0;

  auto node = [&](int k) { return col + plane * map_index(k, A.nk, bk); };
  auto nodeB = [&](int k) { return colB + plane * map_index(k, A.nk, bk); };
  typedef __attribute__((address_space(3))) uint32_t* lds_u32;
  // the ten 4-byte words of the five doubles at src, lane by lane, into rows
  // of `pitch` words starting at LDS byte address base (uniform per wave)
  auto dma_q = [&](const double* src, uint32_t base, int pitch) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(src);
    // earlier reads of the buffer by this wave are complete
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int d = 0; d < 10; ++d)
      asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dword %1, off"
                   :
                   : "s"(base + d * pitch * 4), "v"(w + d)
                   : "memory");
  };
  // five doubles of this lane from such a buffer
  auto lds_q = [&](const uint32_t* row0, int pitch, int lane, Rl out[5]) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const uint64_t lo = row0[2 * v * pitch + lane], hi = row0[(2 * v + 1) * pitch + lane];
      out[v] = (Rl)__builtin_bit_cast(double, (hi << 32) | lo);
    }
  };
  // Q of plane k of an edge thread's second-ring column into sQB
  auto qb_fetch = [&](int k) {
    if constexpr (COMPACT)
      dma_q(reinterpret_cast<const double*>(qin) + 5 * nodeB(k),
            __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_u32)&sQB[0][0]), 64);
  };
  const int laneB = t - NI;   // an edge thread's column in sQB
  // primitives u, v, w, T, p of a column's Q, in the order of the sPr rows
  auto prims_of = [&](const Rl q[5], Rl out[5]) {
    const Prim<Rl> p = primitives(q, gm1, gamma);
    out[0] = p.u;
    out[1] = p.v;
    out[2] = p.w;
    out[3] = p.T;
    out[4] = p.p;
  };
  auto write_prims = [&](int slot, const Rl pr[5]) {
#pragma unroll
    for (int k = 0; k < 5; ++k) sPr[slot][k][c] = pr[k];
  };

  // column registers: Q of planes s-1 (m), s, s+1 (g) and the lead s+2 (l)
  Rl Qm[5], Qs[5], Qg[5], Ql[5];
  Rl nus = 0, sigs = 0;
  double Js = 0.0;
  // Acc carries, from one march step to the next, the in-plane terms of the
  // next plane to be written minus the zeta face flux below it
  Rl Fzs[5] = {0, 0, 0, 0, 0}, Acc[5] = {0, 0, 0, 0, 0};
  double nsum[5] = {0, 0, 0, 0, 0}, nmax[5] = {0, 0, 0, 0, 0};
  double lmax = 0.0;

  // software prefetch, one march step ahead: Q of the next lead plane and
  // the metrics of the next gradient plane
  Rl Qn[5], Mn[9];
  double MJn = 0.0;

  // ring slots: plane k lives in slot (k - kbeg + 3) % 3
  int slot_s = 1, slot_g = 2, slot_l = 0;  // planes kbeg-2, kbeg-1, kbeg
  // primitives of this column at planes s (PrM) and s+1 (PrC), carried in
  // registers when ZREG
  Rl PrM[5] = {0, 0, 0, 0, 0}, PrC[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int v = 0; v < 5; ++v) Qs[v] = Qg[v] = Qn[v] = Qm[v] = 0;
  if (isP) {
    const long long n0 = node(kbeg - 2), n1 = node(kbeg - 1), n2 = node(kbeg);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Qs[v] = (Rl)qin[5 * n0 + v];
      Qg[v] = (Rl)qin[5 * n1 + v];
      Qn[v] = (Rl)qin[5 * n2 + v];
    }
    if (COMPACT || isG) met.load(n1, Mn, MJn);
    prims_of(Qs, PrM);
    prims_of(Qg, PrC);
    if constexpr (!ZREG) {
      write_prims(slot_s, PrM);
      write_prims(slot_g, PrC);
    }
  }
  // the second-ring column's first gradient plane
  if (hasB) qb_fetch(kbeg - 1);

  for (int s = kbeg - 2; s < kend; ++s) {
    // ---- lead plane s+2 (prefetched); prefetch plane s+3 -------------------
#pragma unroll
    for (int v = 0; v < 5; ++v) Ql[v] = Qn[v];
    // the second-ring column's gradient plane s+1, fetched during the
    // previous march step's gradient phase: nothing was issued after it
    if (hasB) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      Rl qb[5], pb[5];
      lds_q(&sQB[0][0], 64, laneB, qb);
      prims_of(qb, pb);
#pragma unroll
      for (int k = 0; k < 5; ++k) sPr[ZREG ? 0 : slot_g][k][cB] = pb[k];
    }
    // The compact form prefetches on every lane and, past the end of the
    // chunk, reloads the last plane it needs: the same loads on every path
    // let the compiler count them when it waits for older loads, instead of
    // assuming they were skipped and waiting for everything in flight.
    if (isP && (COMPACT || s + 3 < kend + 2)) {
      const long long nn = node(COMPACT ? min(s + 3, kend + 1) : s + 3);
#pragma unroll
      for (int v = 0; v < 5; ++v) Qn[v] = (Rl)qin[5 * nn + v];
    }
    // No barrier here: the primitive plane written now (slot_l; the single
    // plane when ZREG) was last read in the previous step's gradient phase
    // (before its second barrier).  The Q, flux, scale and sensor buffers are
    // rewritten only after the next barrier, which every thread reaches after
    // finishing the owned phase.
    Rl(*sQ)[NS] = sQ2[NQB == 2 ? (s - kbeg) & 1 : 0];
    auto write_q = [&]() {
      if (isP) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sQ[v][c] = Qg[v];
      }
      if (hasB) {
        Rl qb[5];
        lds_q(&sQB[0][0], 64, laneB, qb);
#pragma unroll
        for (int v = 0; v < 5; ++v) sQ[v][cB] = qb[v];
      }
    };
    Rl PrL[5] = {0, 0, 0, 0, 0};  // primitives of the lead plane
    if (isP) {
      prims_of(Ql, PrL);
      if constexpr (ZREG) write_prims(0, PrC);  // the gradient plane s+1
      else write_prims(slot_l, PrL);
    }
    if constexpr (NQB == 2) write_q();
    __syncthreads();
    if constexpr (NQB == 1) write_q();

    // ---- gradient plane g = s+1: fluxes, dissipation scales, sensors ------
    Rl Fzg[5] = {0, 0, 0, 0, 0}, sigg = 0, nug = 0;
    double Jg = 0.0;
    // Take the prefetched metrics out of the prefetch registers (into other
    // registers: the early-clobber move keeps the two apart), so that the
    // prefetch for the next plane can land in place and is waited for only
    // where it is used, one march step later.  The compact form does this on
    // every lane, as its lead-plane prefetch.
    // Q(0) (and, in the last stage, the metrics for the next-dt spectral
    // radius) of the node this column updates in the owned phase: the middle
    // stages of the compact form issue these loads as soon as the flux
    // contraction has freed its registers, the other stages and shapes (whose
    // registers do not allow that) just before the second barrier
    const long long ns = node(s);
    constexpr bool Q0_IN_REGS = std::is_same<Rl, double>::value && std::is_same<TIn, double>::value;
    double q0v[5] = {0, 0, 0, 0, 0};
    MT mo[9];
    double moJ = 0.0;
    const bool upd = isI && s >= kbeg && !WRITE_R;  // plane s is updated in this step
    auto update_loads = [&]() {
      if (!(Q0_IN_REGS && q0_is_input)) {
#pragma unroll
        for (int v = 0; v < 5; ++v) q0v[v] = A.q0[5 * ns + v];
      }
      if (LAMMAX && !MET_LDS) met.load(ns, mo, moJ);
    };
    Rl m[9];
    if constexpr (COMPACT) {
#pragma unroll
      for (int k = 0; k < 9; ++k) m[k] = move_apart(Mn[k]);
      Jg = move_apart(MJn);
      met.load(node(min(s + 2, kend)), Mn, MJn);
      // the second-ring column's next gradient plane, straight into LDS
      if (hasB && s + 1 < kend) qb_fetch(s + 2);
    }
    if (isG) {
      if constexpr (!COMPACT) {
#pragma unroll
        for (int k = 0; k < 9; ++k) m[k] = move_apart(Mn[k]);
        Jg = move_apart(MJn);
        if (MET_LDS && t < NI) {
#pragma unroll
          for (int k = 0; k < 9; ++k) sMo[(s + 1) & 1][k][t] = (MT)m[k];
          sMoJ[(s + 1) & 1][t] = Jg;
        }
        if (s + 2 < kend + 1) met.load(node(s + 2), Mn, MJn);
      }
      const Rl J = (Rl)Jg;
      const Rl(*Pg)[NS] = sPr[ZREG ? 0 : slot_g];
      // Every primitive this column needs from the three planes, read in one
      // batch: the memory clobber keeps all the reads ahead of the arithmetic,
      // so their latencies overlap instead of adding up.
      Rl ctr[5], nxm[5], nxp[5], nym[5], nyp[5], nzm[5], nzp[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        nxm[q] = Pg[q][c - 1];
        nxp[q] = Pg[q][c + 1];
        nym[q] = Pg[q][c - P];
        nyp[q] = Pg[q][c + P];
        if constexpr (ZREG) {
          ctr[q] = PrC[q];
          nzm[q] = PrM[q];
          nzp[q] = PrL[q];
        } else {
          ctr[q] = Pg[q][c];
          nzm[q] = sPr[slot_s][q][c];
          nzp[q] = sPr[slot_l][q][c];
        }
      }
      asm volatile("" ::: "memory");
      // chain rule d phi / d x_a = J sum_d S^d_a delta_d phi, with the 1/2 of
      // the centred difference folded into the metric factor
      Rl hm[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) hm[k] = (Rl(0.5) * J) * m[k];
      Rl gr[4][3];  // gr[q][a] = d phi_q / d x_a for phi = u, v, w, T
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const Rl dxi = nxp[q] - nxm[q];
        const Rl deta = nyp[q] - nym[q];
        const Rl dzeta = nzp[q] - nzm[q];
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[q][a] = hm[a] * dxi + hm[3 + a] * deta + hm[6 + a] * dzeta;
      }
      const Rl uu[3] = {ctr[0], ctr[1], ctr[2]};
      const Rl T = ctr[3], p = ctr[4];
      const Rl asnd = sqrt_pos(T);
      const Rl mu = div_pos((Rl)ph.mu_suth * T * asnd, T + (Rl)ph.suth_s);
      // Smagorinsky: |S| = sqrt(2 S_ab S_ab), Delta = J^(-1/3)
      const Rl s01 = gr[0][1] + gr[1][0], s02 = gr[0][2] + gr[2][0], s12 = gr[1][2] + gr[2][1];
      const Rl ss2 = Rl(2) * (gr[0][0] * gr[0][0] + gr[1][1] * gr[1][1] + gr[2][2] * gr[2][2]) +
                     (s01 * s01 + s02 * s02 + s12 * s12);
      const Rl smag = ss2 > Rl(0) ? sqrt_pos(ss2) : Rl(0);
      const Rl delta = inv_cbrt(J);
      const Rl mut = Qg[0] * (Rl)ph.cs2 * delta * delta * smag;
      const Rl kap = (Rl)ph.kap_lam * mu + (Rl)ph.kap_turb * mut;
      const Rl mue = mu + mut;
      const Rl div23 = (Rl(2) / Rl(3)) * (gr[0][0] + gr[1][1] + gr[2][2]);
      // Fhat^d = S^d . (E - V) for each direction d: the inviscid part through
      // the contravariant velocity U^d = S^d . u (rho U, rho u_r U + S^d_r p,
      // (e + p) U), the viscous part through the symmetric stress tensor and
      // the energy column w_a = u_r tau_ra - q_a (q_a = -kappa dT/dx_a).
      // Every multiply-add is an explicit fma and nothing else is contracted,
      // so that each instantiation of this code (shapes, stages, the batch
      // kernel) rounds the same way and their results stay bitwise equal.
      Rl F[3][5], Uc[3];
      {
#pragma clang fp contract(off)
        const Rl txx = mue * fma(Rl(2), gr[0][0], -div23), tyy = mue * fma(Rl(2), gr[1][1], -div23);
        const Rl tzz = mue * fma(Rl(2), gr[2][2], -div23);
        const Rl txy = mue * s01, txz = mue * s02, tyz = mue * s12;
        const Rl tau[3][3] = {{txx, txy, txz}, {txy, tyy, tyz}, {txz, tyz, tzz}};
        Rl wv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          wv[a] = fma(kap, gr[3][a], fma(uu[2], tau[2][a], fma(uu[1], tau[1][a], uu[0] * tau[0][a])));
        const Rl ep = Qg[4] + p;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const Rl sx = m[3 * d], sy = m[3 * d + 1], sz = m[3 * d + 2];
          const Rl U = fma(sz, uu[2], fma(sy, uu[1], sx * uu[0]));
          Uc[d] = U;
          F[d][0] = Qg[0] * U;
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const Rl vis = fma(sz, tau[r][2], fma(sy, tau[r][1], sx * tau[r][0]));
            F[d][1 + r] = fma(Qg[1 + r], U, fma(m[3 * d + r], p, -vis));
          }
          F[d][4] = fma(ep, U, -fma(sz, wv[2], fma(sy, wv[1], sx * wv[0])));
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        sFx[v][c] = F[0][v];
        sFy[v][c] = F[1][v];
        Fzg[v] = F[2][v];
      }
      if constexpr (COMPACT && BASE == 0) {
        if (upd) update_loads();
      }
      // Spectral radii and anisotropic dissipation scales.  With
      // lambda^d = J L^d, L^d = |U^d| + a |S^d|, the scale
      // sigma^d = phi^d lambda^d / J = phi^d L^d (phi depends only on ratios
      // of the radii), so J drops out.
      Rl lam[3];  // L^d
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma clang fp contract(off)
        const Rl sx = m[3 * d], sy = m[3 * d + 1], sz = m[3 * d + 2];
        lam[d] = fma(asnd, sqrt_pos(fma(sz, sz, fma(sy, sy, sx * sx))), fabs(Uc[d]));
      }
      Rl sig[3];
      if (ph.alpha_half) {
        // phi^d L^d = L^d + sum_{e != d} sqrt(L^e L^d) = sqrt(L^d) sum_e sqrt(L^e)
        const Rl r0 = sqrt_pos(lam[0]), r1 = sqrt_pos(lam[1]), r2 = sqrt_pos(lam[2]);
        const Rl rs = r0 + r1 + r2;
        sig[0] = r0 * rs;
        sig[1] = r1 * rs;
        sig[2] = r2 * rs;
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          Rl phi = 1;
#pragma unroll
          for (int e = 0; e < 3; ++e)
            if (e != d) phi += (Rl)pow((double)lam[e] / (double)lam[d], ph.tv_alpha);
          sig[d] = phi * lam[d];
        }
      }
      sSx[c] = sig[0];
      sSy[c] = sig[1];
      sigg = sig[2];
      // pressure sensors |p+ - 2p + p-| / (p+ + 2p + p-) along xi, eta, zeta,
      // the three divisions through one reciprocal of the product of the
      // (positive) denominators
      {
        const Rl ax = fabs(nxp[4] - Rl(2) * p + nxm[4]), bx = nxp[4] + Rl(2) * p + nxm[4];
        const Rl ay = fabs(nyp[4] - Rl(2) * p + nym[4]), by = nyp[4] + Rl(2) * p + nym[4];
        const Rl az = fabs(nzp[4] - Rl(2) * p + nzm[4]), bz = nzp[4] + Rl(2) * p + nzm[4];
        const Rl byz = by * bz, r = rcp_pos(bx * byz);
        sNx[c] = ax * byz * r;
        sNy[c] = ay * (bx * bz) * r;
        nug = az * (bx * by) * r;
      }
    }

    // ---- owned columns, before the barrier: the zeta face between planes s
    // and s+1 needs only the column's registers (and the update loads start
    // here in the shapes other than the compact one)
    const bool own = isI && s >= kbeg - 1;  // plane kbeg-1 is not written
    Rl Hp[5] = {0, 0, 0, 0, 0};
    if (own) {
      if constexpr (!(COMPACT && BASE == 0)) {
        if (upd) update_loads();
      }
      const Rl e2 = k2 * fmax(nus, nug);
      const Rl e4 = fmax(Rl(0), k4 - e2);
      const Rl sg = Rl(0.5) * (sigs + sigg);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const Rl d3 = (Ql[v] - Qm[v]) - Rl(3) * (Qg[v] - Qs[v]);
        Hp[v] = Rl(0.5) * (Fzs[v] + Fzg[v]) - sg * (e2 * (Qg[v] - Qs[v]) - e4 * d3);
      }
    }
    __syncthreads();

    // ---- in-plane terms of plane g, one variable per trip, at column slot cc:
    // variables [vb, ve) rotate into Rr[5 - (ve - vb) .. 4].  FP64: the trips
    // are unrolled (the rotation becomes renaming).  FP32-flux: a rolled loop,
    // which measured faster there; it keeps no register indexed by the trip
    // count.
    constexpr int UNR = sizeof(Rl) == 8 ? 5 : 1;
    typedef __attribute__((address_space(3))) const Rl* lds_ptr;
    auto inplane = [&](int cc, int vb, int ve, Rl Rr[5]) {
      // xi faces cc-1/2 and cc+1/2, eta faces cc-P/2 and cc+P/2 (slots)
      const Rl e2xp = k2 * fmax(sNx[cc], sNx[cc + 1]);
      const Rl e2xm = k2 * fmax(sNx[cc - 1], sNx[cc]);
      const Rl e4xp = fmax(Rl(0), k4 - e2xp), e4xm = fmax(Rl(0), k4 - e2xm);
      const Rl sgxp = Rl(0.5) * (sSx[cc] + sSx[cc + 1]), sgxm = Rl(0.5) * (sSx[cc - 1] + sSx[cc]);
      const Rl e2yp = k2 * fmax(sNy[cc], sNy[cc + P]);
      const Rl e2ym = k2 * fmax(sNy[cc - P], sNy[cc]);
      const Rl e4yp = fmax(Rl(0), k4 - e2yp), e4ym = fmax(Rl(0), k4 - e2ym);
      const Rl sgyp = Rl(0.5) * (sSy[cc] + sSy[cc + P]), sgym = Rl(0.5) * (sSy[cc - P] + sSy[cc]);
#pragma unroll UNR
      for (int v = vb; v < ve; ++v) {
        // The empty asm hides the array base, so that every neighbour
        // access is one base register plus an immediate offset.
        lds_ptr q = (lds_ptr)&sQ[v][cc - 2 * P];
        asm volatile("" : "+v"(q));
        lds_ptr fx = (lds_ptr)&sFx[v][cc - 1];
        asm volatile("" : "+v"(fx));
        lds_ptr fy = (lds_ptr)&sFy[v][cc - P];
        asm volatile("" : "+v"(fy));
        const Rl q0 = q[2 * P];
        const Rl qxp = q[2 * P + 1], qxpp = q[2 * P + 2], qxm = q[2 * P - 1], qxmm = q[2 * P - 2];
        const Rl qyp = q[3 * P], qypp = q[4 * P], qym = q[P], qymm = q[0];
        const Rl fxm = fx[0], fxp = fx[2], fym = fy[0], fyp = fy[2 * P];
        asm volatile("" ::: "memory");  // all reads of the trip issued together
        const Rl dxp = sgxp * (e2xp * (qxp - q0) - e4xp * ((qxpp - qxm) - Rl(3) * (qxp - q0)));
        const Rl dxm = sgxm * (e2xm * (q0 - qxm) - e4xm * ((qxp - qxmm) - Rl(3) * (q0 - qxm)));
        const Rl dyp = sgyp * (e2yp * (qyp - q0) - e4yp * ((qypp - qym) - Rl(3) * (qyp - q0)));
        const Rl dym = sgym * (e2ym * (q0 - qym) - e4ym * ((qyp - qymm) - Rl(3) * (q0 - qym)));
        const Rl cx = Rl(0.5) * (fxp - fxm);
        const Rl cy = Rl(0.5) * (fyp - fym);
#pragma unroll
        for (int r = 0; r < 4; ++r) Rr[r] = Rr[r + 1];
        Rr[4] = (cx + cy) - ((dxp - dxm) + (dyp - dym));
      }
    };
    // sRg buffer written in this march step; the owner reads the other one
    // (written one step earlier: the terms of its plane s)
    const int hbuf = (s - kbeg) & 1;
    if (HELP && isH && s >= kbeg - 1) {
      Rl Rh[5] = {0, 0, 0, 0, 0};
      inplane(ch, NV_OWN, 5, Rh);
#pragma unroll
      for (int k = 0; k < NHV; ++k) sRg[hbuf][k][ch] = Rh[5 - NHV + k];
    }

    // ---- owned columns: residual and update of plane s, in-plane terms of
    // plane g.  The FP64 form updates first: that frees the update's double
    // registers before the unrolled trips.  The FP32-flux form, whose rolled
    // trips give the Q(0) reads of the update more time, updates last.
    constexpr bool UPDATE_FIRST = sizeof(Rl) == 8;
    auto update = [&]() {
      if (HELP && s >= kbeg) {
        // the helper's terms of plane s (its variables) complete the carried sum
#pragma unroll
        for (int k = 0; k < NHV; ++k) Acc[NV_OWN + k] = sRg[hbuf ^ 1][k][c] + Acc[NV_OWN + k];
      }
      if (s >= kbeg) {
        double R[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = Js * (double)(Acc[v] + Hp[v]);
        if (WRITE_R) {
#pragma unroll
          for (int v = 0; v < 5; ++v) qout[5 * ns + v] = (TOut)R[v];
        } else {
          double qn[5];
          // In the first stage the stencil input is Q(0) itself and, in the
          // FP64 form, the column registers hold it exactly: no re-read.
          if (Q0_IN_REGS && q0_is_input) {
#pragma unroll
            for (int v = 0; v < 5; ++v) qn[v] = (double)Qs[v] - adt * R[v];
          } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) qn[v] = q0v[v] - adt * R[v];
          }
#pragma unroll
          for (int v = 0; v < 5; ++v) qout[5 * ns + v] = (TOut)qn[v];
          if constexpr (KEEP_REF) {
            // a node on a far-field reference plane also keeps its double
            // update (see StageArgs::ref)
            {
              const int ci[3] = {ui, uj, s};
              const int nn[3] = {A.ni, A.nj, A.nk};
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                if (A.ref_off[d] < 0) continue;
                const int e = face_e(d), f = face_f(d);
                const long long face = (long long)nn[e] * nn[f], at = ci[e] + (long long)nn[e] * ci[f];
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                  if (ci[d] != (side ? nn[d] - 3 : 2)) continue;
                  double* dst = A.ref + 5 * (A.ref_off[d] + side * face + at);
#pragma unroll
                  for (int v = 0; v < 5; ++v) dst[v] = qn[v];
                }
              }
            }
          }
          if (LAMMAX) {
            if (MET_LDS) {
#pragma unroll
              for (int k = 0; k < 9; ++k) mo[k] = sMo[s & 1][k][t];
              moJ = sMoJ[s & 1][t];
            }
            lmax = max_nan(lmax, lambda_sum(qn, mo, moJ, ph.gamma));
          }
        }
        if (NORMS) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            nsum[v] += R[v] * R[v];
            nmax[v] = max_nan(nmax[v], fabs(R[v]));
          }
        }
      }
    };
    if (own) {
      if constexpr (UPDATE_FIRST) update();
      Rl Rg[5] = {0, 0, 0, 0, 0};
      inplane(c, 0, NV_OWN, Rg);
      // the owner's variables sit in Rg[NHV..4]
      if (HELP) {
#pragma unroll
        for (int v = 0; v < NV_OWN; ++v) Rg[v] = Rg[v + NHV];
      }
      if constexpr (!UPDATE_FIRST) update();
      // Acc: in-plane terms of plane g minus its lower zeta face; with HELP
      // the helper's variables arrive next step, so only -Hp is carried
#pragma unroll
      for (int v = 0; v < 5; ++v) Acc[v] = (v < NV_OWN ? Rg[v] : Rl(0)) - Hp[v];
    }

    // ---- shift the column registers and the ring by one plane ---------------
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Qm[v] = Qs[v];
      Qs[v] = Qg[v];
      Qg[v] = Ql[v];
      Fzs[v] = Fzg[v];
    }
    nus = nug;
    sigs = sigg;
    Js = Jg;
    const int old_s = slot_s;
    slot_s = slot_g;
    slot_g = slot_l;
    slot_l = old_s;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      PrM[k] = PrC[k];
      PrC[k] = PrL[k];
    }
  }

  // ---- deterministic block reductions (fixed tree order) --------------------
  if (NORMS || LAMMAX) {
    // one quantity at a time through the two double rows of sRed
    for (int q = 0; q < (NORMS ? 5 : 0) + (LAMMAX ? 1 : 0); ++q) {
      __syncthreads();
      const bool isnorm = NORMS && q < 5;
      sRed[0][t] = isnorm ? nsum[q] : 0.0;
      sRed[1][t] = isnorm ? nmax[q] : lmax;
      __syncthreads();
      // fold to a power of two, then a fixed binary tree
      constexpr int P2 = (NT & (NT - 1)) == 0 ? NT : (1 << (31 - __builtin_clz(NT)));
      if (P2 != NT) {
        if (t < NT - P2) {
          sRed[0][t] += sRed[0][t + P2];
          sRed[1][t] = max_nan(sRed[1][t], sRed[1][t + P2]);
        }
        __syncthreads();
      }
      for (int st = P2 / 2; st > 0; st >>= 1) {
        if (t < st) {
          sRed[0][t] += sRed[0][t + st];
          sRed[1][t] = max_nan(sRed[1][t], sRed[1][t + st]);
        }
        __syncthreads();
      }
      if (t == 0) {
        if (isnorm) {
          A.norm_part[(long long)lt * 10 + q] = sRed[0][0];
          A.norm_part[(long long)lt * 10 + 5 + q] = sRed[1][0];
        } else {
          A.lam_part[lt] = sRed[1][0];
        }
      }
    }
  }
}


// Waves per SIMD the register allocation must allow: the FP32-flux stages fit
// three (at most 168 VGPRs) except the single-stage form, which carries both
// reductions; the compact FP64 form two (its workgroup has one wave per SIMD,
// and a CU holds two workgroups); the other FP64 shapes leave it to the
// compiler (their 512 threads put two waves on every SIMD).
template <typename Rl, int BX, int BY, int MODE>
constexpr int stage_waves_per_eu() {
  return (sizeof(Rl) == 4 && (MODE & 7) != 3) ? 3 : stage_compact<Rl, BX, BY>() ? 2 : 1;
}

// Single block: one workgroup per tile, tiles spread XCD by XCD.
template <typename Rl, typename TIn, typename TOut, bool MET32, int BX, int BY, int MODE>
__global__ __launch_bounds__((stage_threads<Rl, BX, BY>()))
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<Rl, BX, BY, MODE>()))) void stage_kernel(StageArgs A, const int* __restrict__ flag) {
  if (*flag) return;  // a failed step froze the state
  stage_tile<Rl, TIn, TOut, MET32, BX, BY, MODE, false>(A, xcd_remap(blockIdx.x, gridDim.x));
}

// Many blocks in one persistent launch.  The tiles of all blocks form one
// global list (block b owns [tile_off[b], tile_off[b+1])).  Slot x (the XCD
// that workgroups with blockIdx % 8 == x are dispatched to) takes a
// contiguous share of the list, so neighbouring tiles of a block meet in one
// L2; the workgroups of a slot claim its tiles one at a time, in order, from
// the slot's counter, so a workgroup that drew short tiles takes more of
// them, and every workgroup exits once its slot's share is claimed.  The
// grid is at least kBatchSlots workgroups, so every slot is served.
template <typename Rl, typename TIn, typename TOut, bool MET32, int BX, int BY, int MODE>
__global__ __launch_bounds__((stage_threads<Rl, BX, BY>()))
__attribute__((amdgpu_waves_per_eu(stage_waves_per_eu<Rl, BX, BY, MODE>()))) void stage_batch_kernel(const BlockDesc* __restrict__ desc,
                                                             const int* __restrict__ tile_off,
                                                             BatchCtl* __restrict__ ctl, int stage, int nstages,
                                                             double alpha) {
  __shared__ int sTile;
  const int x = blockIdx.x % kBatchSlots;
  const int nblk = ctl->nblk;
  const int lo = ctl->split[x], hi = ctl->split[x + 1];
  int* next = &ctl->next[stage][x];
  for (;;) {
    __syncthreads();  // the previous tile's LDS readers are done, and sTile is free
    if (threadIdx.x == 0) sTile = lo + atomicAdd(next, 1);
    __syncthreads();
    const int g = sTile;
    if (g >= hi) break;
    // block owning global tile g (uniform over the workgroup)
    int a = 0, b = nblk;
    while (b - a > 1) {
      const int mid = (a + b) >> 1;
      if (tile_off[mid] <= g) a = mid;
      else b = mid;
    }
    const BlockDesc& D = desc[a];
    if (*D.flag) continue;
    StageArgs A;
    const bool last = stage == nstages - 1;
    A.qin = stage == 0 ? (const void*)D.q0 : ((stage - 1) % 2 == 0 ? D.bufA : D.bufB);
    A.qout = last ? (void*)D.q0 : (stage % 2 == 0 ? D.bufA : D.bufB);
    A.q0 = D.q0;
    A.met = D.met;
    A.jac = D.jac;
    A.clock = D.clock;
    A.norm_part = D.norm_part;
    A.lam_part = D.lam_part;
    A.alpha = alpha;
    A.N = D.N;
    A.ni = D.ni;
    A.nj = D.nj;
    A.nk = D.nk;
    A.tiles_i = D.tiles_i;
    A.tiles_j = D.tiles_j;
    A.kchunk = D.kchunk;
    A.nchunks = D.nchunks;
    A.in = D.in;
    A.ph = D.ph;
    stage_tile<Rl, TIn, TOut, MET32, BX, BY, MODE, true>(A, g - tile_off[a]);
  }
}

}  // namespace jz
