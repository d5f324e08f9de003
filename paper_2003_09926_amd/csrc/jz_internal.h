// jz_internal.h -- device-side declarations shared by the HIP sources of the
// jet-LES library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jz {

// Physical constants of one block, derived once on the host from jz_params.
struct Phys {
  double gamma;       // ratio of specific heats
  double gm1;         // gamma - 1
  double mu_suth;     // mu_inf (1 + S): Sutherland numerator with T_inf = 1
  double suth_s;      // S
  double cs2;         // Cs^2
  double kap_lam;     // Cp / Pr
  double kap_turb;    // Cp / Pr_t
  double k2, k4;      // dissipation coefficients
  double tv_alpha;    // anisotropic scaling exponent
  int alpha_half;     // tv_alpha == 0.5 (square-root fast path)
  int pad;
};

// Device-resident clock and diagnostics of one solver (lives in the workspace).
struct Clock {
  double t;          // simulated time
  double dt;         // step size of the next (or current) step
  double lam_max;    // max over nodes of sum_d lambda^d behind dt
  double rms[5];     // first-stage residual norms of the last step
  double linf[5];
  long long steps;
  int flag;          // 0 = healthy; bit 0: non-finite; bit 1: non-positive rho/p/J
  int pad;
};

// Per-step reduction settings read by the finalize kernels.
struct StepCtl {
  double cfl;
  double dt_fixed;
  double inv_n;       // 1 / N
};

// Nodes the residual advances: [lo[d], hi[d]) along each direction.  Bit d of
// bnd is set when direction d ends in physical faces; then its two outermost
// node layers at each end are boundary layers (lo = 2, hi = n - 2), set by
// the boundary conditions, and stencil indices that would leave the block are
// clamped to it instead of wrapped (only boundary-layer nodes, whose residual
// is never used, reach that far).  A periodic direction has lo = 0, hi = n.
struct Interior {
  int lo[3], hi[3];
  int bnd;
};

// Launch shape of the fused stage kernel.
struct Tiling {
  int bx, by;         // workgroup = bx x by threads covering the tile and its 2-node halo
  int ti, tj;         // owned tile = (bx - 4) x (by - 4)
  int kchunk;         // planes marched per workgroup
  int tiles_i, tiles_j, nchunks;
  int nblocks;
};

struct StageArgs {
  const void* qin;      // stencil input Q(k-1), node-major (double or float)
  const double* q0;     // Q(0), node-major doubles (read at the owned node only)
  void* qout;           // Q(k) (or R in residual mode), node-major (double or float)
  const void* met;      // scaled metrics: 10 doubles per node (J last), or 9 floats per node
  const double* jac;    // J per node when the metrics are floats (else unused)
  const Clock* clock;   // dt
  double* norm_part;    // [nblocks][10] first-stage partial sums / maxima
  double* lam_part;     // [nblocks] max sum_d lambda^d of the updated state
  double alpha;         // stage coefficient
  long long N;
  int ni, nj, nk;
  int tiles_i, tiles_j, kchunk, nchunks;
  Interior in;          // tiles and chunks cover [lo, hi) of each direction
  Phys ph;
  // FP32-flux intermediate stages of a block with physical faces: the double
  // update of every node on a far-field reference plane (index 2 or n-3
  // along a bounded direction d) also goes to ref + 5 * (ref_off[d] + side *
  // n_e n_f + c_e + n_e c_f), (e, f) the other two directions in order, so
  // that the boundary rule decides from the double state; NULL otherwise
  double* ref;
  long long ref_off[3];
};

// One member block of a batch: its device buffers, shape and physics.  The
// stage buffers rotate Q0 -> A -> B -> A -> ... -> Q0 as in the single-block
// path.
struct BlockDesc {
  double* q0;
  void* bufA;
  void* bufB;
  const void* met;
  const double* jac;
  Clock* clock;
  double* norm_part;
  double* lam_part;
  int* flag;
  long long N;
  int ni, nj, nk;
  int tiles_i, tiles_j, kchunk, nchunks, ntiles;
  Interior in;
  StepCtl ctl;
  Phys ph;
};

// Work list of a batch, read by its persistent stage launches and kept in
// device memory so that a captured step serves any resident set: the member
// count, the tiles of all members (member by member, each in its logical
// tile order), their split among the XCD slots (slot x takes global tiles
// [split[x], split[x+1]), cut so that the slots get about equal numbers of
// plane steps), and per stage and slot the number of tiles claimed so far
// (the workgroups of a slot claim its tiles in order with an atomic add; the
// finalize launch at the end of a step zeroes the counters for the next).
constexpr int kBatchSlots = 8;
struct BatchCtl {
  int nblk;
  int total;
  int split[kBatchSlots + 1];
  int next[5][kBatchSlots];
};

// One ghost refill of a domain part along direction d: layers [dl0, dl0 + 2)
// of dst take layers [sl0, sl0 + 2) of src, over the whole extent of dst in
// the other two directions (the same as src's); five values per node.
struct HaloJob {
  void* dst;
  const void* src;
  int nd[3], nsrc[3];
  int dl0, sl0;
};

// One sub-block of a domain, for the fixed-order reductions over all of them.
struct DomainSub {
  Clock* clock;
  const double* norm_part;  // [nb_tiles][10] first-stage partials of its last step
  const double* lam_part;   // lambda maxima: per tile, or per lambda_max block
  int* flag;
  int nb_tiles;             // stage-kernel workgroups (tiles) of the sub-block
  int nb_lmax;              // lambda_max_kernel blocks of the sub-block
};

// The two directions of the faces normal to d, the faster first.
__host__ __device__ inline int face_e(int d) { return d == 0 ? 1 : 0; }
__host__ __device__ inline int face_f(int d) { return d == 2 ? 1 : 2; }

// Offset (in nodes) of the reference planes of each bounded direction in the
// FP32-flux reference buffer (-1 for a periodic direction), and the buffer's
// total node count: two planes of n_e x n_f nodes per bounded direction.
__host__ __device__ inline long long ref_layout(const int n[3], int bnd, long long off[3]) {
  long long tot = 0;
  for (int d = 0; d < 3; ++d) {
    off[d] = -1;
    if (!((bnd >> d) & 1)) continue;
    off[d] = tot;
    tot += 2LL * n[face_e(d)] * n[face_f(d)];
  }
  return tot;
}

__host__ __device__ inline int wrap_index(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// index along a direction: periodic wrap, or clamped along a bounded one
__host__ __device__ inline int map_index(int i, int n, bool bounded) {
  if (!bounded) return wrap_index(i, n);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// NaN-propagating maximum (a plain fmax would drop a NaN).
__device__ inline double max_nan(double a, double b) { return (b > a || b != b) ? b : a; }

// FP64 reciprocal and square root for positive, normal arguments: the
// hardware seed refined to about one ulp.  Reciprocal: with e = 1 - y r the
// exact value is r / (1 - e) = r (1 + e + e^2 + ...); the second-order step
// r (1 + e + e^2) leaves a relative error of order e^3, below double rounding
// for a seed good to more than 18 bits.  Square root: one coupled Goldschmidt
// step on g ~ sqrt(x), h ~ 1 / (2 sqrt(x)) from the reciprocal-square-root
// seed, then one Newton correction g + (x - g^2) h.  Both stay within the
// state bar of the FP64 form with orders of magnitude to spare (the residual
// carries far larger rounding from its flux differences).  Non-positive or
// non-finite inputs give NaN/Inf, which the norm and dt checks then report.
__device__ inline double rcp_pos(double y) {
  const double r = __builtin_amdgcn_rcp(y);
  const double e = fma(-y, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

__device__ inline double div_pos(double x, double y) {
  const double r = rcp_pos(y);
  const double q = x * r;
  return fma(fma(-y, q, x), r, q);
}

__device__ inline double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// FP32 counterparts: hardware approximations (about 1 ulp), which is the
// accuracy the FP32-flux form works at
__device__ inline float rcp_pos(float y) { return __builtin_amdgcn_rcpf(y); }
__device__ inline float div_pos(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
__device__ inline float sqrt_pos(float x) { return __builtin_amdgcn_sqrtf(x); }

// sum_d lambda^d at one node: |J S^d . u| + a J |S^d|, the inviscid spectral
// radii in index units that set the CFL time step.  The nine scaled metrics
// come in their stored type (double, or float in the FP32-flux form) and are
// widened here, so every caller computes the same double result.
template <typename M>
__device__ inline double lambda_sum(const double q[5], const M s[9], double J, double gamma) {
  const double rinv = rcp_pos(q[0]);
  const double u = q[1] * rinv, v = q[2] * rinv, w = q[3] * rinv;
  const double p = (gamma - 1.0) * (q[4] - 0.5 * q[0] * (u * u + v * v + w * w));
  const double a = sqrt_pos(gamma * p * rinv);
  double sum = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double sx = (double)s[3 * d], sy = (double)s[3 * d + 1], sz = (double)s[3 * d + 2];
    sum += fabs(J * (sx * u + sy * v + sz * w)) + a * J * sqrt_pos(sx * sx + sy * sy + sz * sz);
  }
  return sum;
}

// Metric views: load the nine scaled metrics of node n in the compute type
// and J in double.
template <bool MET32>
struct MetView;
template <>
struct MetView<false> {  // node-major, 10 doubles per node (J last)
  const double* m;
  const double* jac;
  template <typename Rl>
  __device__ void load(long long n, Rl s[9], double& J) const {
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = (Rl)m[10 * n + k];
    J = m[10 * n + 9];
  }
};
template <>
struct MetView<true> {  // node-major, 9 floats per node; J in its own double array
  const float* m;
  const double* jac;
  template <typename Rl>
  __device__ void load(long long n, Rl s[9], double& J) const {
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = (Rl)m[9 * n + k];
    J = jac[n];
  }
};


// Block index -> logical tile, so that consecutive logical tiles (which are
// neighbours and share halo nodes) land on the same XCD and its L2.
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X.
__device__ inline int xcd_remap(int b, int nb) {
  constexpr int NX = 8;
  const int q = nb / NX, r = nb % NX;
  const int x = b % NX;
  return x * q + (x < r ? x : r) + b / NX;
}

}  // namespace jz
