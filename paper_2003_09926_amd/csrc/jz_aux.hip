// jz_aux.hip -- metric computation, input validation, CFL reduction and the
// per-step finalize kernel of the jet-LES library.
#include <type_traits>
#include "jz_internal.h"

namespace jz {

struct Period {
  double p[9];  // p[3 d + a]: shift of coordinate a when index d wraps forwards
};

namespace {

__device__ inline int floor_div(int a, int n) {
  const int q = a / n;
  return (a % n != 0 && (a < 0)) ? q - 1 : q;
}

struct CoordView {
  const double* X;  // 3 x N coordinates
  long long N;
  int n[3];
  int bnd;          // bit d: direction d bounded (no wrap; one-sided end differences)
  Period P;
  // coordinate a of logical node c, unwrapped across the periodic seams
  __device__ double at(int a, const int c[3]) const {
    const long long idx = (long long)wrap_index(c[0], n[0]) +
                          (long long)n[0] * (wrap_index(c[1], n[1]) + (long long)n[1] * wrap_index(c[2], n[2]));
    double v = X[a * N + idx];
    v += floor_div(c[0], n[0]) * P.p[a];
    v += floor_div(c[1], n[1]) * P.p[3 + a];
    v += floor_div(c[2], n[2]) * P.p[6 + a];
    return v;
  }
};

}  // namespace

// Discretely conservative (Thomas-Lombard) metric set: for cyclic (d, d1, d2)
// and (a, a1, a2),  S^d_a = delta_d2(X_a2 delta_d1 X_a1) - delta_d1(X_a2 delta_d2 X_a1),
// with X_a2 measured from the centre node; J = 1 / det(delta_d X_a).  Because
// the centred differences commute, sum_d delta_d S^d_a vanishes identically,
// which keeps a uniform flow exactly steady on any grid.
//
// Each thread loads the unwrapped coordinates of the 19 nodes the formula
// reaches (the centre, its 6 face and 12 edge neighbours: offsets with at
// most two nonzero components) once, and applies every difference as a
// weighted sum over offsets -1, 0, +1: weights (-1/2, 0, 1/2) inside, and
// along a bounded direction (0, -1, 1) at its first node and (-1, 1, 0) at
// its last (one-sided; they enter only the metrics of the outermost boundary
// layer, i.e. the far-field normal, never the residual of an advanced node).
// MET32 = false: 10 doubles per node; true: 9 floats per node + J in double.
template <bool MET32>
__global__ __launch_bounds__(256) void metrics_tl_kernel(CoordView cv, void* __restrict__ mout,
                                                         double* __restrict__ jac) {
  double* m = (double*)mout;
  float* m32 = (float*)mout;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= cv.N) return;
  const int c[3] = {(int)(n % cv.n[0]), (int)((n / cv.n[0]) % cv.n[1]), (int)(n / ((long long)cv.n[0] * cv.n[1]))};
  // coordinates of the neighbourhood: nb[a][o0 + 3 (o1 + 3 o2) + 13] for offset (o0, o1, o2)
  double nb[3][27];
  for (int o = 0; o < 27; ++o) {
    const int off[3] = {o % 3 - 1, (o / 3) % 3 - 1, o / 9 - 1};
    if (off[0] != 0 && off[1] != 0 && off[2] != 0) continue;  // corners: never reached
    const int e[3] = {c[0] + off[0], c[1] + off[1], c[2] + off[2]};
    for (int a = 0; a < 3; ++a) nb[a][o] = cv.at(a, e);
  }
  // difference weights along each direction at this node, for offsets -1, 0, +1
  double w[3][3];
  for (int d = 0; d < 3; ++d) {
    const bool b = (cv.bnd >> d) & 1;
    const bool first = b && c[d] == 0, last = b && c[d] == cv.n[d] - 1;
    w[d][0] = first ? 0.0 : (last ? -1.0 : -0.5);
    w[d][1] = first ? -1.0 : (last ? 1.0 : 0.0);
    w[d][2] = first ? 1.0 : (last ? 0.0 : 0.5);
  }
  const int stride[3] = {1, 3, 9};
  // difference along d of coordinate a around the node at offset index o
  auto delta = [&](int a, int d, int o) {
    return (w[d][0] * nb[a][o - stride[d]] + w[d][1] * nb[a][o]) + w[d][2] * nb[a][o + stride[d]];
  };
  const int oc = 13;  // the centre
  for (int d = 0; d < 3; ++d) {
    const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
    for (int a = 0; a < 3; ++a) {
      const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
      // outer difference along p of (X_a2 - X_a2(centre)) times the inner
      // difference of X_a1 along q, taken at the nodes o = centre + s e_p
      auto term = [&](int p, int q) {
        double acc = 0.0;
        for (int s = -1; s <= 1; ++s) {
          const int o = oc + s * stride[p];
          acc += w[p][s + 1] * ((nb[a2][o] - nb[a2][oc]) * delta(a1, q, o));
        }
        return acc;
      };
      const double sda = term(d2, d1) - term(d1, d2);
      if (MET32)
        m32[9 * n + 3 * d + a] = (float)sda;
      else
        m[10 * n + 3 * d + a] = sda;
    }
  }
  // J = 1 / det(dX_a / dxi_d), the determinant expanded along its first row
  double M[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) M[a][d] = delta(a, d, oc);
  const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                     M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                     M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  if (MET32)
    jac[n] = 1.0 / det;
  else
    m[10 * n + 9] = 1.0 / det;
}

// flag |= 1 for a non-finite metric, |= 2 for J <= 0
// Nodes on the centreline of a cylindrical mesh (j = 0 when axis_nj > 0, with
// axis_ni = ni, axis_nj = nj) have zero cell volume and no metrics; they are
// never used (the centreline rule sets their state) and are not checked.
__device__ inline bool on_axis(long long n, int axis_ni, int axis_nj) {
  return axis_nj > 0 && (n / axis_ni) % axis_nj == 0;
}

__global__ __launch_bounds__(256) void check_metrics_kernel(const double* __restrict__ m, long long N, int axis_ni,
                                                            int axis_nj, int* __restrict__ flag) {
  int bad = 0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    if (on_axis(n, axis_ni, axis_nj)) continue;
    for (int c = 0; c < 10; ++c)
      if (!isfinite(m[10 * n + c])) bad |= 1;
    if (!(m[10 * n + 9] > 0.0)) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// same checks on the FP32-flux metric storage
__global__ __launch_bounds__(256) void check_met32_kernel(const float* __restrict__ m32, const double* __restrict__ jac,
                                                          long long N, int axis_ni, int axis_nj,
                                                          int* __restrict__ flag) {
  int bad = 0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    if (on_axis(n, axis_ni, axis_nj)) continue;
    for (int c = 0; c < 9; ++c)
      if (!isfinite(m32[9 * n + c])) bad |= 1;
    if (!isfinite(jac[n])) bad |= 1;
    if (!(jac[n] > 0.0)) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// structure-of-arrays metric set (10 x N doubles) -> FP32-flux storage
__global__ __launch_bounds__(256) void soa_to_met32_kernel(const double* __restrict__ src, float* __restrict__ m32,
                                                           double* __restrict__ jac, long long N) {
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    for (int k = 0; k < 9; ++k) m32[9 * n + k] = (float)src[k * N + n];
    jac[n] = src[9 * N + n];
  }
}

// flag |= 1 for a non-finite value, |= 2 for rho <= 0 or p <= 0
__global__ __launch_bounds__(256) void check_state_kernel(const double* __restrict__ q, long long N, double gm1,
                                                          int* __restrict__ flag) {
  int bad = 0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    double v[5];
    for (int c = 0; c < 5; ++c) {
      v[c] = q[5 * n + c];
      if (!isfinite(v[c])) bad |= 1;
    }
    const double p = gm1 * (v[4] - 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0]);
    if (!(v[0] > 0.0) || !(p > 0.0)) bad |= 2;
  }
  if (bad) atomicOr(flag, bad);
}

// per-block max of sum_d lambda^d (grid-stride; max is order-independent).
// Uses the same metric view and arithmetic as the fused last stage, so the
// dt of a restarted run is bitwise the dt of the uninterrupted one.
template <bool MET32>
__global__ __launch_bounds__(256) void lambda_max_kernel(const double* __restrict__ q, MetView<MET32> met,
                                                         long long N, int ni, int nj, Interior in, double gamma,
                                                         double* __restrict__ part) {
  __shared__ double red[256];
  double mx = 0.0;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    if (in.bnd) {  // boundary layers are not advanced and do not set dt
      const int i = (int)(n % ni), j = (int)((n / ni) % nj), k = (int)(n / ((long long)ni * nj));
      if (i < in.lo[0] || i >= in.hi[0] || j < in.lo[1] || j >= in.hi[1] || k < in.lo[2] || k >= in.hi[2]) continue;
    }
    double qq[5], mJ;
    typename std::conditional<MET32, float, double>::type mm[9];
    for (int c = 0; c < 5; ++c) qq[c] = q[5 * n + c];
    met.load(n, mm, mJ);
    mx = max_nan(mx, lambda_sum(qq, mm, mJ, gamma));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = max_nan(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void met32_to_soa_kernel(const float* __restrict__ m32, const double* __restrict__ jac,
                                                           double* __restrict__ dst, long long N) {
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    for (int k = 0; k < 9; ++k) dst[k * N + n] = (double)m32[9 * n + k];
    dst[9 * N + n] = jac[n];
  }
}

namespace {
constexpr int FIN_T = 256;

// Fixed-order reduction of nb partials: thread t folds b = t, t+256, ... in
// order, then a fixed binary tree.  Bitwise reproducible for a given nb.
__device__ double block_sum(const double* part, int stride, int nb, double* red) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += FIN_T) acc += part[(long long)b * stride];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = FIN_T / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_max(const double* part, int stride, int nb, double* red) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += FIN_T) acc = max_nan(acc, part[(long long)b * stride]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = FIN_T / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = max_nan(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double dt_rule(const StepCtl& c, double lmax) { return c.dt_fixed > 0.0 ? c.dt_fixed : c.cfl / lmax; }
}  // namespace

// dt of the first step after a new state: from the lambda partials only
__global__ __launch_bounds__(FIN_T) void finalize_dt_kernel(Clock* clk, const double* __restrict__ lam_part, int nb,
                                                            StepCtl ctl, int* __restrict__ flag) {
  __shared__ double red[FIN_T];
  const double lmax = block_max(lam_part, 1, nb, red);
  if (threadIdx.x == 0) {
    const double dt = dt_rule(ctl, lmax);
    clk->lam_max = lmax;
    clk->dt = dt;
    if (!isfinite(lmax) || !isfinite(dt) || !(dt > 0.0)) *flag |= 1;
  }
}

namespace {
// end of a step: advance the clock by the dt just used, store the first-stage
// norms, and set the next dt from the last stage's lambda partials
__device__ void finalize_step_body(Clock* clk, const double* __restrict__ norm_part,
                                   const double* __restrict__ lam_part, int nb, const StepCtl& ctl,
                                   int* __restrict__ flag, double* red) {
  if (*flag) return;
  double sums[5], maxs[5];
  for (int v = 0; v < 5; ++v) {
    sums[v] = block_sum(norm_part + v, 10, nb, red);
    maxs[v] = block_max(norm_part + 5 + v, 10, nb, red);
  }
  const double lmax = block_max(lam_part, 1, nb, red);
  if (threadIdx.x == 0) {
    bool ok = true;
    for (int v = 0; v < 5; ++v) {
      clk->rms[v] = sqrt(sums[v] * ctl.inv_n);
      clk->linf[v] = maxs[v];
      ok = ok && isfinite(sums[v]) && isfinite(maxs[v]);
    }
    clk->t += clk->dt;
    clk->steps += 1;
    const double dt = dt_rule(ctl, lmax);
    clk->lam_max = lmax;
    clk->dt = dt;
    ok = ok && isfinite(lmax) && isfinite(dt) && dt > 0.0;
    if (!ok) *flag |= 1;
  }
}
}  // namespace

__global__ __launch_bounds__(FIN_T) void finalize_step_kernel(Clock* clk, const double* __restrict__ norm_part,
                                                              const double* __restrict__ lam_part, int nb,
                                                              StepCtl ctl, int* __restrict__ flag) {
  __shared__ double red[FIN_T];
  finalize_step_body(clk, norm_part, lam_part, nb, ctl, flag, red);
}

// one workgroup per member slot of a batch (the table may hold fewer members
// than the launch has workgroups); the first also zeroes the tile counters of
// the stage launches for the next step
__global__ __launch_bounds__(FIN_T) void finalize_batch_kernel(const BlockDesc* __restrict__ desc,
                                                               BatchCtl* __restrict__ ctl) {
  __shared__ double red[FIN_T];
  if (blockIdx.x == 0 && threadIdx.x < 5 * kBatchSlots) (&ctl->next[0][0])[threadIdx.x] = 0;
  if ((int)blockIdx.x >= ctl->nblk) return;
  const BlockDesc& D = desc[blockIdx.x];
  finalize_step_body(D.clock, D.norm_part, D.lam_part, D.ntiles, D.ctl, D.flag, red);
}

// structure-of-arrays (c x N, the ABI layout) <-> node-major (N x c, the
// library's internal layout)
__global__ __launch_bounds__(256) void soa_to_nodes_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                           long long N, int C) {
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x)
    for (int c = 0; c < C; ++c) dst[C * n + c] = src[c * N + n];
}

__global__ __launch_bounds__(256) void nodes_to_soa_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                           long long N, int C) {
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x)
    for (int c = 0; c < C; ++c) dst[c * N + n] = src[C * n + c];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_metrics_tl(const double* X, const double* period9, int ni, int nj, int nk, int bnd, void* m,
                             double* jac, bool met32, hipStream_t st) {
  CoordView cv;
  cv.X = X;
  cv.N = (long long)ni * nj * nk;
  cv.n[0] = ni;
  cv.n[1] = nj;
  cv.n[2] = nk;
  cv.bnd = bnd;
  for (int c = 0; c < 9; ++c) cv.P.p[c] = ((bnd >> (c / 3)) & 1) ? 0.0 : period9[c];
  const long long nb = (cv.N + 255) / 256;
  if (met32)
    hipLaunchKernelGGL(metrics_tl_kernel<true>, dim3((unsigned)nb), dim3(256), 0, st, cv, m, jac);
  else
    hipLaunchKernelGGL(metrics_tl_kernel<false>, dim3((unsigned)nb), dim3(256), 0, st, cv, m, jac);
  return hipGetLastError();
}

static unsigned grid_stride_blocks(long long N) {
  long long nb = (N + 255) / 256;
  return (unsigned)(nb < 2048 ? (nb < 1 ? 1 : nb) : 2048);
}

hipError_t launch_check_metrics(const double* m, long long N, int axis_ni, int axis_nj, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(check_metrics_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, m, N, axis_ni, axis_nj, flag);
  return hipGetLastError();
}

hipError_t launch_check_met32(const float* m32, const double* jac, long long N, int axis_ni, int axis_nj, int* flag,
                              hipStream_t st) {
  hipLaunchKernelGGL(check_met32_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, m32, jac, N, axis_ni, axis_nj,
                     flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// time-averaged statistics (Sec. 6: mean axial velocity and the RMS of its
// fluctuation, here also the pressure), accumulated in FP64 per node
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void stats_accumulate_kernel(const double* __restrict__ q, double* __restrict__ acc,
                                                               long long N, double gamma) {
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const double rho = q[5 * n], mx = q[5 * n + 1], my = q[5 * n + 2], mz = q[5 * n + 3], e = q[5 * n + 4];
    const double u = mx / rho;
    const double p = (gamma - 1.0) * (e - 0.5 * (mx * mx + my * my + mz * mz) / rho);
    acc[4 * n + 0] += u;
    acc[4 * n + 1] += u * u;
    acc[4 * n + 2] += p;
    acc[4 * n + 3] += p * p;
  }
}

// sums -> mean and RMS of the fluctuation, sqrt(max(<x^2> - <x>^2, 0)),
// structure of arrays: out[0..N) mean u, [N..2N) rms u, then mean p, rms p
__global__ __launch_bounds__(256) void stats_finalize_kernel(const double* __restrict__ acc, long long N, double inv_n,
                                                             double* __restrict__ out) {
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
    const double mu = acc[4 * n] * inv_n, mp = acc[4 * n + 2] * inv_n;
    const double vu = acc[4 * n + 1] * inv_n - mu * mu, vp = acc[4 * n + 3] * inv_n - mp * mp;
    out[n] = mu;
    out[N + n] = sqrt(vu > 0.0 ? vu : 0.0);
    out[2 * N + n] = mp;
    out[3 * N + n] = sqrt(vp > 0.0 ? vp : 0.0);
  }
}

// Azimuthal (binned) average of the node statistics over the cross-section
// i: one thread per bin visits the nodes of the plane in the fixed order
// k = 0.., j = 0.. and averages those whose bin index matches, so the result
// does not depend on scheduling.  out[5 b + 0..3] = averaged mean u, rms u,
// mean p, rms p; out[5 b + 4] = node count.
__global__ __launch_bounds__(64) void stats_profile_kernel(const double* __restrict__ soa, long long N, int ni, int nj,
                                                           int nk, int i, const int* __restrict__ bins, int nbins,
                                                           double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double acc[4] = {0, 0, 0, 0};
  long long cnt = 0;
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nj; ++j) {
      if (bins[j + (long long)nj * k] != b) continue;
      const long long n = i + (long long)ni * (j + (long long)nj * k);
      for (int f = 0; f < 4; ++f) acc[f] += soa[f * N + n];
      ++cnt;
    }
  for (int f = 0; f < 4; ++f) out[5 * b + f] = cnt ? acc[f] / (double)cnt : 0.0;
  out[5 * b + 4] = (double)cnt;
}

hipError_t launch_stats_accumulate(const double* q, double* acc, long long N, double gamma, hipStream_t st) {
  hipLaunchKernelGGL(stats_accumulate_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, q, acc, N, gamma);
  return hipGetLastError();
}

hipError_t launch_stats_finalize(const double* acc, long long N, double inv_n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(stats_finalize_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, acc, N, inv_n, out);
  return hipGetLastError();
}

hipError_t launch_stats_profile(const double* soa, long long N, int ni, int nj, int nk, int i, const int* bins,
                                int nbins, double* out, hipStream_t st) {
  hipLaunchKernelGGL(stats_profile_kernel, dim3((nbins + 63) / 64), dim3(64), 0, st, soa, N, ni, nj, nk, i, bins, nbins,
                     out);
  return hipGetLastError();
}

hipError_t launch_soa_to_met32(const double* src, float* m32, double* jac, long long N, hipStream_t st) {
  hipLaunchKernelGGL(soa_to_met32_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, src, m32, jac, N);
  return hipGetLastError();
}

hipError_t launch_check_state(const double* q, long long N, double gm1, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(check_state_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, q, N, gm1, flag);
  return hipGetLastError();
}

hipError_t launch_soa_to_nodes(const double* src, double* dst, long long N, int C, hipStream_t st) {
  hipLaunchKernelGGL(soa_to_nodes_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, src, dst, N, C);
  return hipGetLastError();
}

hipError_t launch_nodes_to_soa(const double* src, double* dst, long long N, int C, hipStream_t st) {
  hipLaunchKernelGGL(nodes_to_soa_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, src, dst, N, C);
  return hipGetLastError();
}

int lambda_max_blocks(long long N) { return (int)grid_stride_blocks(N); }

hipError_t launch_lambda_max(const double* q, const void* met, const double* jac, bool met32, long long N,
                             const int n[3], Interior in, double gamma, double* part, hipStream_t st) {
  if (met32) {
    MetView<true> mv;
    mv.m = (const float*)met;
    mv.jac = jac;
    hipLaunchKernelGGL(lambda_max_kernel<true>, dim3(grid_stride_blocks(N)), dim3(256), 0, st, q, mv, N, n[0], n[1], in,
                       gamma, part);
  } else {
    MetView<false> mv;
    mv.m = (const double*)met;
    mv.jac = jac;
    hipLaunchKernelGGL(lambda_max_kernel<false>, dim3(grid_stride_blocks(N)), dim3(256), 0, st, q, mv, N, n[0], n[1], in,
                       gamma, part);
  }
  return hipGetLastError();
}

hipError_t launch_met32_to_soa(const float* m32, const double* jac, double* dst, long long N, hipStream_t st) {
  hipLaunchKernelGGL(met32_to_soa_kernel, dim3(grid_stride_blocks(N)), dim3(256), 0, st, m32, jac, dst, N);
  return hipGetLastError();
}

hipError_t launch_finalize_dt(Clock* clk, const double* lam_part, int nb, StepCtl ctl, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(FIN_T), 0, st, clk, lam_part, nb, ctl, flag);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const BlockDesc* desc, BatchCtl* ctl, int slots, hipStream_t st) {
  hipLaunchKernelGGL(finalize_batch_kernel, dim3(slots), dim3(FIN_T), 0, st, desc, ctl);
  return hipGetLastError();
}

hipError_t launch_finalize_step(Clock* clk, const double* norm_part, const double* lam_part, int nb, StepCtl ctl,
                                int* flag, hipStream_t st) {
  hipLaunchKernelGGL(finalize_step_kernel, dim3(1), dim3(FIN_T), 0, st, clk, norm_part, lam_part, nb, ctl, flag);
  return hipGetLastError();
}


// Clock and failure flag of a run that starts afresh: time 0, step 0, no
// failure (a kernel rather than a memset or a host copy, so that the work can
// be captured in a graph).
__global__ void reset_clock_kernel(Clock* __restrict__ clk, int* __restrict__ flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    Clock c;
    c.t = 0.0;
    c.dt = 0.0;
    c.lam_max = 0.0;
    for (int v = 0; v < 5; ++v) c.rms[v] = c.linf[v] = 0.0;
    c.steps = 0;
    c.flag = 0;
    c.pad = 0;
    *clk = c;
    *flag = 0;
  }
}

// Clock and flag as 14 doubles: t, dt of the next step, rms[5], linf[5],
// steps, flag.
__global__ void export_clock_kernel(const Clock* __restrict__ clk, const int* __restrict__ flag,
                                    double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    out[0] = clk->t;
    out[1] = clk->dt;
    for (int v = 0; v < 5; ++v) {
      out[2 + v] = clk->rms[v];
      out[7 + v] = clk->linf[v];
    }
    out[12] = (double)clk->steps;
    out[13] = (double)*flag;
  }
}

hipError_t launch_reset_clock(Clock* clk, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(reset_clock_kernel, dim3(1), dim3(64), 0, st, clk, flag);
  return hipGetLastError();
}

hipError_t launch_export_clock(const Clock* clk, const int* flag, double* out, hipStream_t st) {
  hipLaunchKernelGGL(export_clock_kernel, dim3(1), dim3(64), 0, st, clk, flag, out);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// domains: one block split into sub-blocks with two ghost layers along each
// split direction (the decomposition of Sec. 4.1, exchanged as in Sec. 4.3)
// ---------------------------------------------------------------------------
// Two node layers of direction d, all positions across it: dst layers dl0,
// dl0 + 1 <- src layers sl0, sl0 + 1 (node-major, 5 values per node).  The
// two blocks have the same extents across d.
// Every ghost refill of one exchange pass in one launch: workgroup row y
// serves job y (rows beyond a job's size return at once).
template <typename T>
__global__ __launch_bounds__(256) void halo_jobs_kernel(const HaloJob* __restrict__ jobs, int d) {
  const HaloJob& J = jobs[blockIdx.y];
  const int e = face_e(d), f = face_f(d);
  const long long face = (long long)J.nd[e] * J.nd[f];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (d == 0) {
    // along xi the two ghost layers of a row are neighbouring nodes, ten
    // contiguous values: ten consecutive threads copy them
    if (t >= face * 10) return;
    const long long row = t / 10;
    const int q = (int)(t % 10);
    const int j = (int)(row % J.nd[1]), k = (int)(row / J.nd[1]);
    const long long id = J.dl0 + (long long)J.nd[0] * (j + (long long)J.nd[1] * k);
    const long long is = J.sl0 + (long long)J.nsrc[0] * (j + (long long)J.nsrc[1] * k);
    static_cast<T*>(J.dst)[5 * id + q] = static_cast<const T*>(J.src)[5 * is + q];
    return;
  }
  // along eta or zeta the face planes are contiguous: one thread per value,
  // the five values of a node, then the face nodes, then the layer
  if (t >= 2 * face * 5) return;
  const int v = (int)(t % 5);
  const int layer = (int)((t / 5) / face);
  const long long r = (t / 5) % face;
  int c[3];
  c[e] = (int)(r % J.nd[e]);
  c[f] = (int)(r / J.nd[e]);
  c[d] = J.dl0 + layer;
  const long long id = c[0] + (long long)J.nd[0] * (c[1] + (long long)J.nd[1] * c[2]);
  c[d] = J.sl0 + layer;
  const long long is = c[0] + (long long)J.nsrc[0] * (c[1] + (long long)J.nsrc[1] * c[2]);
  static_cast<T*>(J.dst)[5 * id + v] = static_cast<const T*>(J.src)[5 * is + v];
}

hipError_t launch_halo_jobs(const HaloJob* jobs, int njobs, bool is_float, int d, long long max_count,
                            hipStream_t st) {
  if (njobs < 1) return hipSuccess;
  const dim3 grid((unsigned)((max_count + 255) / 256), (unsigned)njobs);
  if (is_float)
    hipLaunchKernelGGL(halo_jobs_kernel<float>, grid, dim3(256), 0, st, jobs, d);
  else
    hipLaunchKernelGGL(halo_jobs_kernel<double>, grid, dim3(256), 0, st, jobs, d);
  return hipGetLastError();
}

// dt of a domain's first step after a new state: the maximum of sum_d
// lambda^d over every sub-block's advanced nodes (the lambda_max partials),
// written to every sub-block's clock.
__global__ __launch_bounds__(FIN_T) void domain_dt_kernel(const DomainSub* __restrict__ sub, int P, StepCtl ctl) {
  __shared__ double red[FIN_T];
  double lmax = 0.0;
  for (int p = 0; p < P; ++p) lmax = max_nan(lmax, block_max(sub[p].lam_part, 1, sub[p].nb_lmax, red));
  if (threadIdx.x == 0) {
    const double dt = dt_rule(ctl, lmax);
    const bool bad = !isfinite(lmax) || !isfinite(dt) || !(dt > 0.0);
    for (int p = 0; p < P; ++p) {
      sub[p].clock->lam_max = lmax;
      sub[p].clock->dt = dt;
      if (bad) *sub[p].flag |= 1;
    }
  }
}

// First level of a domain step's reductions, one workgroup per sub-block:
// its first-stage norm sums and maxima and its largest spectral radius, each
// in the sub-block's fixed tile order, to part_red[p][0..10].
__global__ __launch_bounds__(FIN_T) void domain_part_reduce_kernel(const DomainSub* __restrict__ sub,
                                                                   double* __restrict__ part_red) {
  __shared__ double red[FIN_T];
  const DomainSub& S = sub[blockIdx.x];
  double* out = part_red + 11 * blockIdx.x;
  for (int v = 0; v < 5; ++v) {
    const double sv = block_sum(S.norm_part + v, 10, S.nb_tiles, red);
    const double mv = block_max(S.norm_part + 5 + v, 10, S.nb_tiles, red);
    if (threadIdx.x == 0) {
      out[v] = sv;
      out[5 + v] = mv;
    }
  }
  const double lm = block_max(S.lam_part, 1, S.nb_tiles, red);
  if (threadIdx.x == 0) out[10] = lm;
}

// End of a domain step: the first-stage norms over all sub-blocks (their
// first-level results added in sub-block order), the clock advanced by the dt
// just used, and the next dt from the last stage's lambda maxima of all
// sub-blocks -- the same values in every sub-block's clock.
__global__ __launch_bounds__(FIN_T) void domain_finalize_kernel(const DomainSub* __restrict__ sub, int P,
                                                                StepCtl ctl, BatchCtl* __restrict__ work,
                                                                const double* __restrict__ part_red) {
  // the tile counters of the batched stage launches, for the next step
  if (work && threadIdx.x < 5 * kBatchSlots) (&work->next[0][0])[threadIdx.x] = 0;
  if (threadIdx.x != 0) return;
  for (int p = 0; p < P; ++p)
    if (*sub[p].flag) return;  // a failed step froze the state
  // second level: the parts' results in part order
  double sums[5] = {0, 0, 0, 0, 0}, maxs[5] = {0, 0, 0, 0, 0}, lmax = 0.0;
  for (int p = 0; p < P; ++p) {
    for (int v = 0; v < 5; ++v) {
      sums[v] += part_red[11 * p + v];
      maxs[v] = max_nan(maxs[v], part_red[11 * p + 5 + v]);
    }
    lmax = max_nan(lmax, part_red[11 * p + 10]);
  }
  bool ok = isfinite(lmax);
  for (int v = 0; v < 5; ++v) ok = ok && isfinite(sums[v]) && isfinite(maxs[v]);
  const double dt = dt_rule(ctl, lmax);
  ok = ok && isfinite(dt) && dt > 0.0;
  for (int p = 0; p < P; ++p) {
    Clock* c = sub[p].clock;
    for (int v = 0; v < 5; ++v) {
      c->rms[v] = sqrt(sums[v] * ctl.inv_n);
      c->linf[v] = maxs[v];
    }
    c->t += c->dt;
    c->steps += 1;
    c->lam_max = lmax;
    c->dt = dt;
    if (!ok) *sub[p].flag |= 1;
  }
}

hipError_t launch_domain_dt(const DomainSub* sub, int P, StepCtl ctl, hipStream_t st) {
  hipLaunchKernelGGL(domain_dt_kernel, dim3(1), dim3(FIN_T), 0, st, sub, P, ctl);
  return hipGetLastError();
}

hipError_t launch_domain_finalize(const DomainSub* sub, int P, StepCtl ctl, BatchCtl* work, double* part_red,
                                  hipStream_t st) {
  hipLaunchKernelGGL(domain_part_reduce_kernel, dim3(P), dim3(FIN_T), 0, st, sub, part_red);
  hipLaunchKernelGGL(domain_finalize_kernel, dim3(1), dim3(FIN_T), 0, st, sub, P, ctl, work,
                     (const double*)part_red);
  return hipGetLastError();
}

}  // namespace jz
