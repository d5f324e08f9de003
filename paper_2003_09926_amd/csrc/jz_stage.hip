// jz_stage.hip -- fused residual + Runge-Kutta stage kernel (FP64).
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
// Every global access uses periodically wrapped indices, so the halo is the
// block's own periodic image (standing in for the neighbour-rank ghost
// layers of Sec. 4.3).  Inside the library Q is stored node-major (the five
// conserved variables of a node contiguous, 40 B) and the metric set likewise
// (10 doubles, 80 B per node): one address per node and array, and a
// wavefront still reads one contiguous span per plane row.
#include "jz_internal.h"

namespace jz {

namespace {

struct Prim {
  double u, v, w, T, p;
};

// FP64 reciprocal and square root for positive, normal arguments: hardware
// seed refined by Newton (reciprocal) and Goldschmidt (square root)
// iterations to full double precision.  Non-positive or non-finite inputs
// give NaN/Inf, which the norm and dt checks then report.
__device__ inline double rcp_pos(double y) {
  double r = __builtin_amdgcn_rcp(y);
  double e = fma(-y, r, 1.0);
  r = fma(r, e, r);
  e = fma(-y, r, 1.0);
  return fma(r, e, r);
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
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

__device__ inline Prim primitives(const double q[5], double gm1, double gamma) {
  Prim r;
  const double rinv = rcp_pos(q[0]);
  r.u = q[1] * rinv;
  r.v = q[2] * rinv;
  r.w = q[3] * rinv;
  r.p = gm1 * (q[4] - 0.5 * q[0] * (r.u * r.u + r.v * r.v + r.w * r.w));
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

__device__ inline double sensor(double pm, double p0, double pp) {
  return div_pos(fabs(pp - 2.0 * p0 + pm), pp + 2.0 * p0 + pm);
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

}  // namespace

// MODE bit 0: accumulate norms of R (first stage)
// MODE bit 1: max of sum_d lambda^d of the updated state (last stage -> next dt)
// MODE bit 2: write R itself instead of the stage update
template <int BX, int BY, int MODE>
__global__ __launch_bounds__(BX* BY) void stage_fp64(StageArgs A, const int* __restrict__ flag) {
  constexpr int NT = BX * BY;
  constexpr int TI = BX - 4, TJ = BY - 4;
  constexpr bool NORMS = (MODE & 1) != 0;
  constexpr bool LAMMAX = (MODE & 2) != 0;
  constexpr bool WRITE_R = (MODE & 4) != 0;
  static_assert((NT & (NT - 1)) == 0, "workgroup size must be a power of two");
  static_assert(TI * TJ + 4 * TI + 4 * TJ + 4 <= NT, "tile roles exceed the workgroup");

  // plane buffers (structure of arrays, one slot per thread/column)
  __shared__ double sPr[3][5][NT];     // ring of three planes of u, v, w, T, p
  __shared__ double sQ[5][NT];         // Q of the gradient plane
  __shared__ double sF[10][NT];        // Fhat^xi (rows 0-4) and Fhat^eta (rows 5-9) of the gradient plane
  double(*sFx)[NT] = sF;
  double(*sFy)[NT] = sF + 5;
  __shared__ double sSx[NT], sSy[NT];  // sigma^xi, sigma^eta
  __shared__ double sNx[NT], sNy[NT];  // pressure sensor along xi, eta

  if (*flag) return;  // a failed step froze the state

  const Phys ph = A.ph;
  const int nb = gridDim.x;
  const int lt = xcd_remap(blockIdx.x, nb);
  const int tile_i = lt % A.tiles_i;
  const int rest = lt / A.tiles_i;
  const int tile_j = rest % A.tiles_j;
  const int chunk = rest / A.tiles_j;
  const int i0 = tile_i * TI, j0 = tile_j * TJ;
  const int kbeg = chunk * A.kchunk;
  const int kend = min(kbeg + A.kchunk, A.nk);

  const int t = threadIdx.x;
  int tx, ty;
  const int role = tile_role<TI, TJ>(t, tx, ty);
  const int c = tx + BX * ty;                     // LDS slot of this column
  const int ui = i0 - 2 + tx, uj = j0 - 2 + ty;  // unwrapped column indices
  const long long col = (long long)wrap_index(ui, A.ni) + (long long)A.ni * wrap_index(uj, A.nj);
  const long long plane = (long long)A.ni * A.nj;
  const bool isP = role <= 2;                     // supplies primitives and Q
  const bool isG = role <= 1;                     // computes fluxes
  const bool isI = role == 0 && ui < A.ni && uj < A.nj;  // owns (writes) its column

  const double* __restrict__ qin = A.qin;
  const double* __restrict__ met = A.met;
  const double dt = A.clock->dt;
  const double adt = A.alpha * dt;

  auto node = [&](int k) { return col + plane * wrap_index(k, A.nk); };
  auto put_prims = [&](int slot, const double q[5]) {
    if (!isP) return;
    const Prim p = primitives(q, ph.gm1, ph.gamma);
    sPr[slot][0][c] = p.u;
    sPr[slot][1][c] = p.v;
    sPr[slot][2][c] = p.w;
    sPr[slot][3][c] = p.T;
    sPr[slot][4][c] = p.p;
  };

  // column registers: Q of planes s-1 (m), s, s+1 (g) and the lead s+2 (l)
  double Qm[5], Qs[5], Qg[5], Ql[5];
  double nus = 0.0, sigs = 0.0, Js = 0.0;
  double Fzs[5] = {0, 0, 0, 0, 0}, Hm[5] = {0, 0, 0, 0, 0}, Rin[5] = {0, 0, 0, 0, 0};
  double nsum[5] = {0, 0, 0, 0, 0}, nmax[5] = {0, 0, 0, 0, 0};
  double lmax = 0.0;

  // software prefetch, one march step ahead: Q of the next lead plane and
  // the metrics of the next gradient plane
  double Qn[5], Mn[10];

  // ring slots: plane k lives in slot (k - kbeg + 3) % 3
  int slot_s = 1, slot_g = 2, slot_l = 0;  // planes kbeg-2, kbeg-1, kbeg
#pragma unroll
  for (int v = 0; v < 5; ++v) Qs[v] = Qg[v] = Qn[v] = Qm[v] = 0.0;
  if (isP) {
    const long long n0 = node(kbeg - 2), n1 = node(kbeg - 1), n2 = node(kbeg);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Qs[v] = qin[5 * n0 + v];
      Qg[v] = qin[5 * n1 + v];
      Qn[v] = qin[5 * n2 + v];
    }
    if (isG) {
#pragma unroll
      for (int k = 0; k < 10; ++k) Mn[k] = met[10 * n1 + k];
    }
    put_prims(slot_s, Qs);
    put_prims(slot_g, Qg);
  }

  for (int s = kbeg - 2; s < kend; ++s) {
    // ---- lead plane s+2 (prefetched); prefetch plane s+3 -------------------
#pragma unroll
    for (int v = 0; v < 5; ++v) Ql[v] = Qn[v];
    if (isP && s + 3 < kend + 2) {
      const long long nn = node(s + 3);
#pragma unroll
      for (int v = 0; v < 5; ++v) Qn[v] = qin[5 * nn + v];
    }
    __syncthreads();  // the previous step's readers of slot_l, sQ, sF*, sS*, sN* are done
    put_prims(slot_l, Ql);
    if (isP) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sQ[v][c] = Qg[v];
    }
    __syncthreads();

    // ---- gradient plane g = s+1: fluxes, dissipation scales, sensors ------
    double Fzg[5] = {0, 0, 0, 0, 0}, sigg = 0.0, nug = 0.0, Jg = 0.0;
    if (isG) {
      double m[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) m[k] = Mn[k];
      if (s + 2 < kend + 1) {
        const long long nm = node(s + 2);
#pragma unroll
        for (int k = 0; k < 10; ++k) Mn[k] = met[10 * nm + k];
      }
      const double J = m[9];
      Jg = J;
      const double (*Pg)[NT] = sPr[slot_g];
      // chain rule d phi / d x_a = J sum_d S^d_a delta_d phi, with the 1/2 of
      // the centred difference folded into the metric factor
      double hm[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) hm[k] = (0.5 * J) * m[k];
      double gr[4][3];  // gr[q][a] = d phi_q / d x_a for phi = u, v, w, T
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double dxi = Pg[q][c + 1] - Pg[q][c - 1];
        const double deta = Pg[q][c + BX] - Pg[q][c - BX];
        const double dzeta = sPr[slot_l][q][c] - sPr[slot_s][q][c];
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[q][a] = hm[a] * dxi + hm[3 + a] * deta + hm[6 + a] * dzeta;
      }
      const double uu[3] = {Pg[0][c], Pg[1][c], Pg[2][c]};
      const double T = Pg[3][c], p = Pg[4][c];
      const double asnd = sqrt_pos(T);
      const double mu = div_pos(ph.mu_suth * T * asnd, T + ph.suth_s);
      // Smagorinsky: |S| = sqrt(2 S_ab S_ab), Delta = J^(-1/3)
      const double s01 = gr[0][1] + gr[1][0], s02 = gr[0][2] + gr[2][0], s12 = gr[1][2] + gr[2][1];
      const double ss2 = 2.0 * (gr[0][0] * gr[0][0] + gr[1][1] * gr[1][1] + gr[2][2] * gr[2][2]) +
                         (s01 * s01 + s02 * s02 + s12 * s12);
      const double smag = ss2 > 0.0 ? sqrt_pos(ss2) : 0.0;
      const double delta = inv_cbrt(J);
      const double mut = Qg[0] * ph.cs2 * delta * delta * smag;
      const double kap = ph.kap_lam * mu + ph.kap_turb * mut;
      const double mue = mu + mut;
      const double div23 = (2.0 / 3.0) * (gr[0][0] + gr[1][1] + gr[2][2]);
      // Fhat^d = sum_a S^d_a (E_a - V_a), one Cartesian column a at a time
      double F[3][5];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        double ta[3];  // column a of the stress tensor
#pragma unroll
        for (int r = 0; r < 3; ++r) ta[r] = mue * (gr[r][a] + gr[a][r] - (r == a ? div23 : 0.0));
        double ev[5];
        ev[0] = Qg[0] * uu[a];
#pragma unroll
        for (int r = 0; r < 3; ++r) ev[1 + r] = Qg[1 + r] * uu[a] + (r == a ? p : 0.0) - ta[r];
        ev[4] = (Qg[4] + p) * uu[a] - (uu[0] * ta[0] + uu[1] * ta[1] + uu[2] * ta[2] + kap * gr[3][a]);
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int v = 0; v < 5; ++v) F[d][v] = (a == 0) ? m[3 * d] * ev[v] : fma(m[3 * d + a], ev[v], F[d][v]);
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        sFx[v][c] = F[0][v];
        sFy[v][c] = F[1][v];
        Fzg[v] = F[2][v];
      }
      // spectral radii and anisotropic dissipation scales
      double lam[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double sx = m[3 * d], sy = m[3 * d + 1], sz = m[3 * d + 2];
        lam[d] = fabs(J * (sx * uu[0] + sy * uu[1] + sz * uu[2])) + asnd * J * sqrt_pos(sx * sx + sy * sy + sz * sz);
      }
      double sig[3];
      const double jinv = rcp_pos(J);
      if (ph.alpha_half) {
        // phi^d lambda^d = lambda^d + sum_{e != d} sqrt(lambda^e lambda^d)
        const double r0 = sqrt_pos(lam[0]), r1 = sqrt_pos(lam[1]), r2 = sqrt_pos(lam[2]);
        const double rs = (r0 + r1 + r2) * jinv;
        sig[0] = r0 * rs;
        sig[1] = r1 * rs;
        sig[2] = r2 * rs;
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          double phi = 1.0;
#pragma unroll
          for (int e = 0; e < 3; ++e)
            if (e != d) phi += pow(lam[e] / lam[d], ph.tv_alpha);
          sig[d] = phi * lam[d] * jinv;
        }
      }
      sSx[c] = sig[0];
      sSy[c] = sig[1];
      sigg = sig[2];
      sNx[c] = sensor(Pg[4][c - 1], p, Pg[4][c + 1]);
      sNy[c] = sensor(Pg[4][c - BX], p, Pg[4][c + BX]);
      nug = sensor(sPr[slot_s][4][c], p, sPr[slot_l][4][c]);
    }
    __syncthreads();

    // ---- owned columns: in-plane terms of plane g, zeta face, residual of s ----
    if (isI) {
      double Rg[5];
      {
        // xi faces t-1/2 and t+1/2, eta faces t-BX/2 and t+BX/2
        const double e2xp = ph.k2 * fmax(sNx[c], sNx[c + 1]);
        const double e2xm = ph.k2 * fmax(sNx[c - 1], sNx[c]);
        const double e4xp = fmax(0.0, ph.k4 - e2xp), e4xm = fmax(0.0, ph.k4 - e2xm);
        const double sgxp = 0.5 * (sSx[c] + sSx[c + 1]), sgxm = 0.5 * (sSx[c - 1] + sSx[c]);
        const double e2yp = ph.k2 * fmax(sNy[c], sNy[c + BX]);
        const double e2ym = ph.k2 * fmax(sNy[c - BX], sNy[c]);
        const double e4yp = fmax(0.0, ph.k4 - e2yp), e4ym = fmax(0.0, ph.k4 - e2ym);
        const double sgyp = 0.5 * (sSy[c] + sSy[c + BX]), sgym = 0.5 * (sSy[c - BX] + sSy[c]);
#pragma unroll 1
        for (int v = 0; v < 5; ++v) {
          const double q0 = sQ[v][c];
          const double qxp = sQ[v][c + 1], qxpp = sQ[v][c + 2], qxm = sQ[v][c - 1], qxmm = sQ[v][c - 2];
          const double qyp = sQ[v][c + BX], qypp = sQ[v][c + 2 * BX], qym = sQ[v][c - BX], qymm = sQ[v][c - 2 * BX];
          const double dxp = sgxp * (e2xp * (qxp - q0) - e4xp * ((qxpp - qxm) - 3.0 * (qxp - q0)));
          const double dxm = sgxm * (e2xm * (q0 - qxm) - e4xm * ((qxp - qxmm) - 3.0 * (q0 - qxm)));
          const double dyp = sgyp * (e2yp * (qyp - q0) - e4yp * ((qypp - qym) - 3.0 * (qyp - q0)));
          const double dym = sgym * (e2ym * (q0 - qym) - e4ym * ((qyp - qymm) - 3.0 * (q0 - qym)));
          const double cx = 0.5 * (sFx[v][c + 1] - sFx[v][c - 1]);
          const double cy = 0.5 * (sFy[v][c + BX] - sFy[v][c - BX]);
          Rg[v] = (cx + cy) - ((dxp - dxm) + (dyp - dym));
        }
      }
      if (s >= kbeg - 1) {
        // zeta face between planes s and s+1
        const double e2 = ph.k2 * fmax(nus, nug);
        const double e4 = fmax(0.0, ph.k4 - e2);
        const double sg = 0.5 * (sigs + sigg);
        double Hp[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const double d3 = (Ql[v] - Qm[v]) - 3.0 * (Qg[v] - Qs[v]);
          Hp[v] = 0.5 * (Fzs[v] + Fzg[v]) - sg * (e2 * (Qg[v] - Qs[v]) - e4 * d3);
        }
        if (s >= kbeg) {
          const long long ns = node(s);
          double R[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) R[v] = Js * (Rin[v] + (Hp[v] - Hm[v]));
          if (WRITE_R) {
#pragma unroll
            for (int v = 0; v < 5; ++v) A.qout[5 * ns + v] = R[v];
          } else {
            double qn[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              qn[v] = A.q0[5 * ns + v] - adt * R[v];
              A.qout[5 * ns + v] = qn[v];
            }
            if (LAMMAX) {
              double m[10];
#pragma unroll
              for (int k = 0; k < 10; ++k) m[k] = met[10 * ns + k];
              lmax = max_nan(lmax, lambda_sum(qn, m, ph.gamma));
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
#pragma unroll
        for (int v = 0; v < 5; ++v) Hm[v] = Hp[v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) Rin[v] = Rg[v];
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
  }

  // ---- deterministic block reductions (fixed tree order) --------------------
  if (NORMS || LAMMAX) {
    double* red = &sF[0][0];  // reuse the 10 x NT flux buffer
    __syncthreads();
    if (NORMS) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        red[v * NT + t] = nsum[v];
        red[(5 + v) * NT + t] = nmax[v];
      }
    }
    if (LAMMAX) sSx[t] = lmax;
    __syncthreads();
    for (int st = NT / 2; st > 0; st >>= 1) {
      if (t < st) {
        if (NORMS) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            red[v * NT + t] += red[v * NT + t + st];
            red[(5 + v) * NT + t] = max_nan(red[(5 + v) * NT + t], red[(5 + v) * NT + t + st]);
          }
        }
        if (LAMMAX) sSx[t] = max_nan(sSx[t], sSx[t + st]);
      }
      __syncthreads();
    }
    if (t == 0) {
      if (NORMS)
        for (int v = 0; v < 10; ++v) A.norm_part[(long long)blockIdx.x * 10 + v] = red[v * NT];
      if (LAMMAX) A.lam_part[blockIdx.x] = sSx[0];
    }
  }
}

// ---------------------------------------------------------------------------
// host-side launcher
// ---------------------------------------------------------------------------
template <int BX, int BY>
static hipError_t launch_shape(const StageArgs& a, const int* flag, int mode, int nblocks, hipStream_t st) {
  const dim3 grid(nblocks), block(BX * BY);
  switch (mode) {
    case 0: hipLaunchKernelGGL((stage_fp64<BX, BY, 0>), grid, block, 0, st, a, flag); break;
    case 1: hipLaunchKernelGGL((stage_fp64<BX, BY, 1>), grid, block, 0, st, a, flag); break;
    case 2: hipLaunchKernelGGL((stage_fp64<BX, BY, 2>), grid, block, 0, st, a, flag); break;
    case 3: hipLaunchKernelGGL((stage_fp64<BX, BY, 3>), grid, block, 0, st, a, flag); break;
    case 4: hipLaunchKernelGGL((stage_fp64<BX, BY, 4>), grid, block, 0, st, a, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Supported workgroup shapes (bx x by threads); the tile is (bx-4) x (by-4).
bool stage_shape_supported(int bx, int by) {
  return (bx == 32 && by == 16) || (bx == 64 && by == 8) || (bx == 16 && by == 32) ||
         (bx == 32 && by == 8) || (bx == 16 && by == 16);
}

hipError_t launch_stage_fp64(const StageArgs& a, const int* flag, int mode, int bx, int by, int nblocks,
                             hipStream_t st) {
  if (bx == 32 && by == 16) return launch_shape<32, 16>(a, flag, mode, nblocks, st);
  if (bx == 64 && by == 8) return launch_shape<64, 8>(a, flag, mode, nblocks, st);
  if (bx == 16 && by == 32) return launch_shape<16, 32>(a, flag, mode, nblocks, st);
  if (bx == 32 && by == 8) return launch_shape<32, 8>(a, flag, mode, nblocks, st);
  if (bx == 16 && by == 16) return launch_shape<16, 16>(a, flag, mode, nblocks, st);
  return hipErrorInvalidValue;
}

}  // namespace jz
