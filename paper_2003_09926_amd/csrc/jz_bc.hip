// jz_bc.hip -- physical boundary conditions of a block (Sec. 3, boundary
// conditions): supersonic inflow at the jet exit (the state there is held),
// a far field computed from Riemann invariants, and the centreline of a
// cylindrical mesh (extrapolation from the adjacent ring and a fixed-order
// azimuthal average, Sec. 3 and the reproducibility rule of Sec. 4.3).  They are applied to the
// boundary layers of a stage output after the stage kernel has advanced the
// interior, one launch per bounded direction in the order xi, eta, zeta.
#include <type_traits>
#include "jz_internal.h"

namespace jz {

namespace {

struct BcArgs {
  int n[3];
  int d;                 // direction whose boundary layers this launch sets
  int bc[6];             // face types (0 periodic, 1 inflow, 2 far field, 3 centreline)
  double gamma;
  double mach_inf;       // free-stream velocity along x in ambient sound speeds
  long long count;       // 4 layers x n_e x n_f nodes
  const double* ref;     // double states of the reference planes (float stage states), or NULL
  long long ref_off;     // offset of direction d's two planes in ref (nodes)
};

// Far-field state from the one-dimensional characteristics normal to the face
// (outward unit normal nh).  Along the normal, u_n + 2a/(gamma-1) travels out
// of the block and u_n - 2a/(gamma-1) into it: the face takes the first from
// the interior state qi and the second from the free stream (rho = 1,
// u = (mach_inf, 0, 0), p = 1/gamma, a = 1), which fixes u_n and a there.
// The other two characteristic quantities, entropy and tangential velocity,
// are carried by the flow: the face takes them from the side the flow comes
// from (the "upwind state" w).  With the entropy of w, rho a^(2/(1-gamma)) is
// constant along the isentrope, so the face density is rho_w (a_b / a_w)^(2 /
// (gamma - 1)).  A supersonic normal flow carries all five quantities from
// its upwind side, whose conserved state the face then takes as it is.
__device__ void farfield_state(double g, double mach_inf, const double qi[5], const double nh[3], double qb[5]) {
  const double gm1 = g - 1.0;
  // interior primitives
  const double rinv = 1.0 / qi[0];
  double vi[3], ke_i = 0.0;
  for (int a = 0; a < 3; ++a) {
    vi[a] = qi[1 + a] * rinv;
    ke_i += qi[1 + a] * vi[a];
  }
  const double p_i = gm1 * (qi[4] - 0.5 * ke_i);
  const double c_i = sqrt(g * p_i * rinv);
  const double un_i = vi[0] * nh[0] + vi[1] * nh[1] + vi[2] * nh[2];
  const double un_inf = mach_inf * nh[0];  // free-stream normal velocity, sound speed 1
  if (un_i >= c_i) {  // supersonic outflow
    for (int v = 0; v < 5; ++v) qb[v] = qi[v];
    return;
  }
  if (un_i <= -c_i) {  // supersonic inflow
    qb[0] = 1.0;
    qb[1] = mach_inf;
    qb[2] = 0.0;
    qb[3] = 0.0;
    qb[4] = 1.0 / (g * gm1) + 0.5 * mach_inf * mach_inf;
    return;
  }
  const double out_inv = un_i + 2.0 * c_i / gm1;  // leaves through the face
  const double in_inv = un_inf - 2.0 / gm1;       // enters from the free stream
  const double un_b = 0.5 * (out_inv + in_inv);
  const double c_b = 0.25 * gm1 * (out_inv - in_inv);
  // the upwind state w: density, sound speed, velocity and its normal part
  const bool outflow = un_b > 0.0;
  const double rho_w = outflow ? qi[0] : 1.0;
  const double c_w = outflow ? c_i : 1.0;
  const double vw[3] = {outflow ? vi[0] : mach_inf, outflow ? vi[1] : 0.0, outflow ? vi[2] : 0.0};
  const double un_w = outflow ? un_i : un_inf;
  const double rho_b = rho_w * pow(c_b / c_w, 2.0 / gm1);
  double ke_b = 0.0;
  qb[0] = rho_b;
  for (int a = 0; a < 3; ++a) {
    const double vb = vw[a] + (un_b - un_w) * nh[a];  // tangential part of w, normal part from the invariants
    qb[1 + a] = rho_b * vb;
    ke_b += vb * vb;
  }
  qb[4] = rho_b * c_b * c_b / (g * gm1) + 0.5 * rho_b * ke_b;  // p = rho a^2 / gamma
}

// Centreline: the average over all azimuths of ring j = 2 of each conserved
// variable at each axial station i, summed in the order k = 0, 1, ..., nk-1
// (the fixed order every axis node uses).  A workgroup takes AXS stations:
// its threads stage the ring values of 256 azimuths at a time in LDS (one
// azimuth per thread, the stations' 5 AXS values contiguous in memory), then
// one thread per (station, variable) adds them in azimuth order.
constexpr int AXS = 4;     // axial stations per workgroup
constexpr int AXK = 256;   // azimuths staged per pass (= threads)
template <typename T>
__global__ __launch_bounds__(AXK) void axis_mean_kernel(const T* __restrict__ q, int ni, int nj, int nk,
                                                        double* __restrict__ mean) {
  __shared__ double buf[AXK][5 * AXS];
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * AXS;
  const int ns = min(AXS, ni - i0);  // stations of this workgroup
  const long long row = (long long)ni * nj;
  const T* __restrict__ ring = q + 5 * (i0 + 2LL * ni);  // (i0, 2, 0)
  double acc = 0.0;
  for (int k0 = 0; k0 < nk; k0 += AXK) {
    const int cnt = min(AXK, nk - k0);
    if (t < cnt) {
      const T* __restrict__ p = ring + 5 * (k0 + t) * row;
      for (int u = 0; u < 5 * ns; ++u) buf[t][u] = (double)p[u];
    }
    __syncthreads();
    if (t < 5 * ns) {
      for (int kk = 0; kk < cnt; ++kk) acc += buf[kk][t];
    }
    __syncthreads();
  }
  if (t < 5 * ns) mean[5 * i0 + t] = acc / (double)nk;
}

// One thread per boundary-layer node of direction d.  Nodes read as
// references (index 2 or n-3 along d, all azimuths of ring 2 for the
// centreline) are never written by the same launch.
template <typename T, bool MET32>
__global__ __launch_bounds__(256) void bc_kernel(T* __restrict__ q, const double* __restrict__ q0, MetView<MET32> met,
                                                 const double* __restrict__ axis_mean, BcArgs b) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b.count) return;
  // Consecutive threads take neighbouring nodes in memory: along xi (the
  // contiguous index) on the eta and zeta faces, the two adjacent layers of
  // one row on the xi faces.
  const int d = b.d, e = d == 0 ? 1 : 0, f = d == 2 ? 1 : 2;  // in-face directions, e the faster
  int layer;
  long long r;
  if (d == 0) {
    layer = (int)(t % 4);
    r = t / 4;
  } else {
    const long long face = (long long)b.n[e] * b.n[f];
    layer = (int)(t / face);
    r = t % face;
  }
  int c[3];
  c[d] = layer < 2 ? layer : b.n[d] - 4 + layer;  // 0, 1, n-2, n-1
  c[e] = (int)(r % b.n[e]);
  c[f] = (int)(r / b.n[e]);
  const bool lo = layer < 2;
  const long long node = c[0] + (long long)b.n[0] * (c[1] + (long long)b.n[1] * c[2]);
  // supersonic inflow: a node in the layers of any inflow face is held at
  // its Q(0) value, whichever other faces it belongs to
  bool held = false;
  for (int x = 0; x < 3; ++x) {
    if (b.bc[2 * x] == 0) continue;
    if ((c[x] < 2 && b.bc[2 * x] == 1) || (c[x] > b.n[x] - 3 && b.bc[2 * x + 1] == 1)) held = true;
  }
  if (held) {
    if ((const void*)q != (const void*)q0) {
      for (int v = 0; v < 5; ++v) q[5 * node + v] = (T)q0[5 * node + v];
    }
    return;
  }
  if ((lo ? b.bc[2 * d] : b.bc[2 * d + 1]) == 3) {
    // centreline (eta- face, d = 1): ring j = 1 extrapolated from the first
    // advanced ring j = 2 (zeroth order, per azimuth); axis nodes j = 0 set
    // to the average over all azimuths of that ring (axis_mean_kernel, one
    // fixed-order sum per axial station: every axis node of one i gets the
    // bitwise same value)
    double acc[5];
    if (c[1] == 1) {
      const long long src = node + b.n[0];  // (i, 2, k)
      for (int v = 0; v < 5; ++v) acc[v] = (double)q[5 * src + v];
    } else {
      for (int v = 0; v < 5; ++v) acc[v] = axis_mean[5 * c[0] + v];
    }
    for (int v = 0; v < 5; ++v) q[5 * node + v] = (T)acc[v];
    return;
  }
  int cr[3] = {c[0], c[1], c[2]};
  cr[d] = lo ? 2 : b.n[d] - 3;
  const long long ref = cr[0] + (long long)b.n[0] * (cr[1] + (long long)b.n[1] * cr[2]);
  double qi[5], qb[5], nh[3];
  // the stage kernel kept double updates for the reference nodes it advanced;
  // a reference node inside another direction's boundary layers (along the
  // edges and corners of the block) has the value an earlier pass of this
  // stage set, in the stage state itself
  bool advanced = true;
  for (int x = 0; x < 3; ++x)
    if (x != d && b.bc[2 * x] != 0 && (cr[x] < 2 || cr[x] > b.n[x] - 3)) advanced = false;
  if (b.ref && advanced) {
    // a float stage state: the rule decides from the double update the stage
    // kept for the reference plane, as for a double state
    const long long o = b.ref_off + (lo ? 0 : 1) * (long long)b.n[e] * b.n[f] + cr[e] + (long long)b.n[e] * cr[f];
    for (int v = 0; v < 5; ++v) qi[v] = b.ref[5 * o + v];
  } else {
    for (int v = 0; v < 5; ++v) qi[v] = (double)q[5 * ref + v];
  }
  typename std::conditional<MET32, float, double>::type sm[9];
  double J;
  met.load(node, sm, J);
  double len = 0.0;
  for (int a = 0; a < 3; ++a) {
    nh[a] = J * (double)sm[3 * d + a];  // grad xi_d
    len += nh[a] * nh[a];
  }
  len = sqrt(len);
  for (int a = 0; a < 3; ++a) nh[a] = (lo ? -nh[a] : nh[a]) / len;
  farfield_state(b.gamma, b.mach_inf, qi, nh, qb);
  for (int v = 0; v < 5; ++v) q[5 * node + v] = (T)qb[v];
}

template <typename T, bool MET32>
hipError_t launch_bc_typed(T* q, const double* q0, const void* met, const double* jac, const int n[3],
                           const int bc[6], double gamma, double mach_inf, double* axis_mean, const double* ref,
                           hipStream_t st) {
  long long ref_off[3];
  int bnd = 0;
  for (int d = 0; d < 3; ++d)
    if (bc[2 * d] != 0) bnd |= 1 << d;
  ref_layout(n, bnd, ref_off);
  MetView<MET32> mv;
  mv.m = (decltype(mv.m))met;
  mv.jac = jac;
  for (int d = 0; d < 3; ++d) {
    if (bc[2 * d] == 0) continue;
    BcArgs b;
    for (int e = 0; e < 3; ++e) b.n[e] = n[e];
    b.d = d;
    for (int f = 0; f < 6; ++f) b.bc[f] = bc[f];
    b.gamma = gamma;
    b.mach_inf = mach_inf;
    b.count = 4LL * n[(d + 1) % 3] * n[(d + 2) % 3];
    b.ref = ref;
    b.ref_off = ref_off[d];
    if (d == 1 && bc[2] == 3) {
      // the centreline means, from ring 2 as the xi pass left it
      if (!axis_mean) return hipErrorInvalidValue;
      const int mb = (n[0] + AXS - 1) / AXS;
      hipLaunchKernelGGL((axis_mean_kernel<T>), dim3(mb), dim3(AXK), 0, st, (const T*)q, n[0], n[1], n[2], axis_mean);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    const long long blocks = (b.count + 255) / 256;
    hipLaunchKernelGGL((bc_kernel<T, MET32>), dim3((unsigned)blocks), dim3(256), 0, st, q, q0, mv,
                       (const double*)axis_mean, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// Boundary conditions on the stage state q (node-major; double, or float when
// q_float), with inflow layers taken from Q(0) = q0.  axis_mean: scratch of
// 5 x n[0] doubles, required when the eta- face is the centreline.  ref: for
// a float stage state, the double states of the far-field reference planes
// (ref_layout) the stage kept, from which the far-field rule then decides
// (NULL: the rule reads q).  No-op for a periodic block.
hipError_t launch_bc(void* q, bool q_float, const double* q0, const void* met, const double* jac, bool met32,
                     const int n[3], const int bc[6], double gamma, double mach_inf, double* axis_mean,
                     const double* ref, hipStream_t st) {
  if (q_float) {
    if (met32) return launch_bc_typed<float, true>((float*)q, q0, met, jac, n, bc, gamma, mach_inf, axis_mean, ref, st);
    return launch_bc_typed<float, false>((float*)q, q0, met, jac, n, bc, gamma, mach_inf, axis_mean, ref, st);
  }
  if (met32) return launch_bc_typed<double, true>((double*)q, q0, met, jac, n, bc, gamma, mach_inf, axis_mean, ref, st);
  return launch_bc_typed<double, false>((double*)q, q0, met, jac, n, bc, gamma, mach_inf, axis_mean, ref, st);
}

}  // namespace jz
