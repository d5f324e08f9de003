// jetles_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, FP64 CPU oracle of the jet-LES hot path: the residual of the
// filtered compressible Navier-Stokes equations on a periodic structured
// curvilinear block, and the explicit five-stage Runge-Kutta step built on it.
// Only the tests, the smoke check and the CPU-baseline leg of the benchmark
// load it.  It shares no code, header, table or helper with the HIP library.
//
// Every loop runs over whole fields, one step of the method at a time, in the
// order the paper states them:
//   * conservation laws, Favre-filtered variables          Sec. 3, Eq. (les)
//   * total energy and equation of state                   Sec. 3, energy/EOS
//   * heat flux q_j = -kappa dT/dx_j, kappa = mu Cp / Pr   Sec. 3, Eq. (q_mod)
//   * Sutherland viscosity                                 Sec. 3, Eq. (sutherland)
//   * Stokes stress tensor                                 Sec. 3, Eq. (tau_mod)
//   * dQ/dt = -RHS, inviscid E and viscous F fluxes        Sec. 3, Eqs. (vec-les), (con-prop)
//   * curvilinear form, 2nd-order centred differences with
//     anisotropic scalar artificial dissipation            Sec. 3, closing paragraph
//   * explicit five-stage Runge-Kutta, full residual in
//     every stage                                          Sec. 3; Sec. 4.2 and its flow chart
//   * five-point dissipation stencil, two ghost layers     Sec. 4.3
//   * physical boundaries: supersonic inflow at the jet
//     exit, far field from Riemann invariants, centreline
//     of a cylindrical mesh (extrapolation + azimuthal
//     average in a fixed order)                            Sec. 3, boundary conditions; Sec. 4.3
// Points the paper leaves open (subgrid closure, dissipation constants, RK
// coefficients, time-step rule, viscous stencil, metric form, scales) follow
// the readings listed with the design notes; each is a field of jzo_params.
//
// Parity status: the metric, residual and step functions are pinned by
// closed forms and invariants in tests/test_oracle_pins.py (free-stream
// preservation, discrete conservation, isentropic vortex, second-order
// convergence, shear-wave and entropy-wave decay factors, Smagorinsky closed
// form, mirror symmetry), the viscous closure and the shock branch of the
// dissipation in tests/test_oracle_closure_pins.py (heat conduction, the
// -2/3 div u stress, the viscous work in the energy flux, each against its
// Fourier-mode closed form; a periodic Sod pair against the exact Riemann
// solution with the fourth-difference coefficient clamped at the shocks)
// and the boundary treatment in tests/test_oracle_bc_pins.py
// (Riemann-invariant identities, free-stream preservation and conservation
// on bounded blocks, transparency to an outgoing acoustic pulse).  The
// numerical values of the open constants are "parity unpinned" against the
// paper, which prints none.
#include <cmath>
#include <cstddef>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>

extern "C" {

typedef struct {
  double gamma;        // ratio of specific heats
  double prandtl;      // molecular Prandtl number (0.72, Sec. 3)
  double prandtl_t;    // turbulent Prandtl number of the subgrid heat flux
  double mach_j;       // jet Mach number = jet velocity in ambient sound speeds
  double re_d;         // Reynolds number on the jet diameter (mu_inf = mach_j / re_d)
  double sutherland_s; // Sutherland constant over the reference temperature
  double cs;           // Smagorinsky constant
  double k2, k4;       // second- and fourth-difference dissipation coefficients
  double tv_alpha;     // exponent of the anisotropic (Turkel-Vatsa) scaling
  double cfl;          // Courant number of the global time step
  double dt_fixed;     // > 0: use this time step instead of the CFL rule
  double rk_alpha[5];  // stage coefficients Q(k) = Q(0) - a_k dt R(Q(k-1))
  int n_stages;
  // boundary type of the faces xi-, xi+, eta-, eta+, zeta-, zeta+:
  // 0 periodic, 1 supersonic inflow (state held), 2 far field (Riemann
  // invariants), 3 centreline (eta- only, zeta periodic: eta = radius from
  // the axis, zeta = azimuth)
  int bc[6];
  double mach_inf;     // far-field stream velocity along x, in ambient sound speeds
} jzo_params;

int jzo_params_default(jzo_params* p) {
  if (!p) return -1;
  p->gamma = 1.4;
  p->prandtl = 0.72;
  p->prandtl_t = 0.9;
  p->mach_j = 1.4;
  p->re_d = 1.0e5;
  p->sutherland_s = 110.4 / 288.15;
  p->cs = 0.17;
  p->k2 = 0.25;
  p->k4 = 1.0 / 64.0;
  p->tv_alpha = 0.5;
  p->cfl = 0.5;
  p->dt_fixed = 0.0;
  p->rk_alpha[0] = 1.0 / 4.0;
  p->rk_alpha[1] = 1.0 / 6.0;
  p->rk_alpha[2] = 3.0 / 8.0;
  p->rk_alpha[3] = 1.0 / 2.0;
  p->rk_alpha[4] = 1.0;
  p->n_stages = 5;
  for (int f = 0; f < 6; ++f) p->bc[f] = 0;
  p->mach_inf = 0.0;
  return 0;
}

}  // extern "C"

namespace {

// A block is periodic along each direction unless its faces there carry
// physical boundaries; then the two outermost node layers at each end are
// boundary layers (set by the boundary conditions, never advanced by the
// residual) and the nodes between them are the interior.
struct Block {
  int n[3];
  long N;
  bool bnd[3];  // direction bounded by physical faces
  Block(int ni, int nj, int nk, const int* bc = nullptr) {
    n[0] = ni; n[1] = nj; n[2] = nk;
    N = (long)ni * nj * nk;
    for (int d = 0; d < 3; ++d) bnd[d] = bc && bc[2 * d] != 0;
  }
  static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  // index along d: periodic wrap, or clamped to the block along a bounded
  // direction (only reached by stencils of boundary-layer nodes, whose
  // residual is never used)
  int idx(int i, int d) const {
    if (!bnd[d]) return wrap(i, n[d]);
    return i < 0 ? 0 : (i >= n[d] ? n[d] - 1 : i);
  }
  long at(int i, int j, int k) const {
    return idx(i, 0) + (long)n[0] * (idx(j, 1) + (long)n[1] * idx(k, 2));
  }
  bool interior(int i, int j, int k) const {
    const int c[3] = {i, j, k};
    for (int d = 0; d < 3; ++d)
      if (bnd[d] && (c[d] < 2 || c[d] > n[d] - 3)) return false;
    return true;
  }
  long n_interior() const {
    long r = 1;
    for (int d = 0; d < 3; ++d) r *= bnd[d] ? n[d] - 4 : n[d];
    return r;
  }
  // linear index of the neighbour `off` steps along direction d
  long nb(int i, int j, int k, int d, int off) const {
    int c[3] = {i, j, k};
    c[d] += off;
    return at(c[0], c[1], c[2]);
  }
};

static int floordiv(int a, int n) {
  int q = a / n;
  if ((a % n) != 0 && ((a < 0) != (n < 0))) --q;
  return q;
}

// ---------------------------------------------------------------------------
// Geometry: metric terms and Jacobian of the curvilinear transformation
// (Sec. 3 closing paragraph; computed once after reading the mesh, Sec. 4.2).
// ---------------------------------------------------------------------------
struct Coords {
  const Block& b;
  const double* X[3];
  double P[3][3];  // P[d][a]: shift of coordinate a when index d wraps by +n_d
  // coordinate a of logical node c (indices may lie outside the block),
  // unwrapped across the periodic seams
  double get(int a, const int c[3]) const {
    double v = X[a][b.at(c[0], c[1], c[2])];
    for (int d = 0; d < 3; ++d) v += floordiv(c[d], b.n[d]) * P[d][a];
    return v;
  }
};

// Difference of a node function g along d at logical node c: centred, or
// one-sided (first order) at the end nodes of a bounded direction, where
// the centred stencil would leave the block.
template <class G>
static double diff(const Block& b, const G& g, const int c[3], int d) {
  int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
  if (b.bnd[d] && c[d] == 0) {
    cp[d] += 1;
    return g(cp) - g(c);
  }
  if (b.bnd[d] && c[d] == b.n[d] - 1) {
    cm[d] -= 1;
    return g(c) - g(cm);
  }
  cp[d] += 1;
  cm[d] -= 1;
  return 0.5 * (g(cp) - g(cm));
}

// Thomas-Lombard conservative metrics,
//   S^d_a = delta_d2( x_a2 delta_d1 x_a1 ) - delta_d1( x_a2 delta_d2 x_a1 )
// with (d, d1, d2) and (a, a1, a2) cyclic, x_a2 taken relative to the centre
// node (an exact identity that limits roundoff); J^-1 = det of the matrix of
// coordinate differences.  Output m[3 d + a] = S^d_a, m[9] = J.  Along a
// bounded direction the differences at the two end nodes are one-sided.
static void metrics_tl(const Block& b, const double* const X[3], const double* period9, double* m) {
  Coords C{b, {X[0], X[1], X[2]}, {{0}}};
  for (int d = 0; d < 3; ++d)
    for (int a = 0; a < 3; ++a) C.P[d][a] = b.bnd[d] ? 0.0 : period9[3 * d + a];
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b.n[2]; ++k)
    for (int j = 0; j < b.n[1]; ++j)
      for (int i = 0; i < b.n[0]; ++i) {
        const int c[3] = {i, j, k};
        const long p = b.at(i, j, k);
        for (int d = 0; d < 3; ++d) {
          const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
          for (int a = 0; a < 3; ++a) {
            const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
            const double xc = C.get(a2, c);
            auto xa1 = [&](const int* e) { return C.get(a1, e); };
            auto h1 = [&](const int* e) { return (C.get(a2, e) - xc) * diff(b, xa1, e, d1); };
            auto h2 = [&](const int* e) { return (C.get(a2, e) - xc) * diff(b, xa1, e, d2); };
            m[(3 * d + a) * b.N + p] = diff(b, h1, c, d2) - diff(b, h2, c, d1);
          }
        }
        double M[3][3];  // M[a][d] = d x_a / d xi_d
        for (int a = 0; a < 3; ++a) {
          auto xa = [&](const int* e) { return C.get(a, e); };
          for (int d = 0; d < 3; ++d) M[a][d] = diff(b, xa, c, d);
        }
        const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                           M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        m[9 * b.N + p] = 1.0 / det;
      }
}

}  // namespace

extern "C" {

int jzo_metrics_tl(int ni, int nj, int nk, const double* x, const double* y, const double* z,
                   const double* period9, double* m) {
  if (ni < 1 || nj < 1 || nk < 1 || !x || !y || !z || !period9 || !m) return -1;
  Block b(ni, nj, nk);
  const double* X[3] = {x, y, z};
  metrics_tl(b, X, period9, m);
  return 0;
}

// The same on a block whose faces carry the boundary types bc[6] (see
// jzo_params): directions with physical faces get one-sided end differences.
int jzo_metrics_tl_bc(int ni, int nj, int nk, const double* x, const double* y, const double* z,
                      const double* period9, const int* bc, double* m) {
  if (ni < 1 || nj < 1 || nk < 1 || !x || !y || !z || !period9 || !m || !bc) return -1;
  const int n[3] = {ni, nj, nk};
  for (int d = 0; d < 3; ++d)
    if ((bc[2 * d] != 0) != (bc[2 * d + 1] != 0) || (bc[2 * d] != 0 && n[d] < 5)) return -1;
  Block b(ni, nj, nk, bc);
  const double* X[3] = {x, y, z};
  metrics_tl(b, X, period9, m);
  return 0;
}

}  // extern "C"

namespace {

// All per-node fields of one residual evaluation.
struct Fields {
  long N;
  std::vector<double> rho, u, v, w, p, T, a;   // primitives
  std::vector<double> g;                        // 12 x N: d(u,v,w,T)/d(x,y,z)
  std::vector<double> mu, mut;                  // molecular and subgrid viscosity
  std::vector<double> F;                        // 15 x N: contravariant flux F^d_v
  std::vector<double> lam;                      // 3 x N spectral radii lambda^d
  std::vector<double> sig;                      // 3 x N dissipation scale sigma^d
  std::vector<double> nu;                       // 3 x N pressure sensor nu^d
  explicit Fields(long n)
      : N(n), rho(n), u(n), v(n), w(n), p(n), T(n), a(n), g(12 * n), mu(n), mut(n), F(15 * n),
        lam(3 * n), sig(3 * n), nu(3 * n) {}
};

// Steps 1-8 of the residual, leaving every intermediate field in `f`.
static void node_fields(const Block& b, const jzo_params& P, const double* m, const double* q,
                        Fields& f) {
  const long N = b.N;
  const double gam = P.gamma;
  const double cp = 1.0 / (gam - 1.0);          // Cp with R = 1/gamma (T_inf = 1)
  const double mu_inf = (P.re_d > 0.0 && std::isfinite(P.re_d)) ? P.mach_j / P.re_d : 0.0;

  // primitives: u_i = (rho u_i)/rho; p from the total energy; T = gamma p / rho
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    const double rho = q[n];
    const double u = q[N + n] / rho, v = q[2 * N + n] / rho, w = q[3 * N + n] / rho;
    const double p = (gam - 1.0) * (q[4 * N + n] - 0.5 * rho * (u * u + v * v + w * w));
    const double T = gam * p / rho;
    f.rho[n] = rho; f.u[n] = u; f.v[n] = v; f.w[n] = w; f.p[n] = p; f.T[n] = T;
    f.a[n] = std::sqrt(T);
  }

  // velocity and temperature gradients by the chain rule
  //   d phi / d x_a = J sum_d S^d_a delta_d phi
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b.n[2]; ++k)
    for (int j = 0; j < b.n[1]; ++j)
      for (int i = 0; i < b.n[0]; ++i) {
        const long n = b.at(i, j, k);
        const double J = m[9 * N + n];
        const double* phi[4] = {f.u.data(), f.v.data(), f.w.data(), f.T.data()};
        for (int s = 0; s < 4; ++s) {
          double dd[3];
          for (int d = 0; d < 3; ++d)
            dd[d] = 0.5 * (phi[s][b.nb(i, j, k, d, +1)] - phi[s][b.nb(i, j, k, d, -1)]);
          for (int a = 0; a < 3; ++a) {
            double acc = 0.0;
            for (int d = 0; d < 3; ++d) acc += m[(3 * d + a) * N + n] * dd[d];
            f.g[(3 * s + a) * N + n] = J * acc;
          }
        }
      }

  // viscosities, stresses, heat flux, Cartesian and contravariant fluxes
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    const double J = m[9 * N + n];
    const double T = f.T[n];
    // Sutherland, with T_inf = T_0 = 1
    const double mu = mu_inf * std::pow(T, 1.5) * (1.0 + P.sutherland_s) / (T + P.sutherland_s);
    double du[3][3];  // du[a][b] = d u_a / d x_b
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) du[a][c] = f.g[(3 * a + c) * N + n];
    // Smagorinsky: |S| = sqrt(2 S_ab S_ab), Delta = J^(-1/3)
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        const double sab = 0.5 * (du[a][c] + du[c][a]);
        ss += sab * sab;
      }
    const double smag = std::sqrt(2.0 * ss);
    const double delta = std::cbrt(1.0 / J);
    const double mut = f.rho[n] * (P.cs * delta) * (P.cs * delta) * smag;
    f.mu[n] = mu;
    f.mut[n] = mut;
    const double kap = cp * mu / P.prandtl + cp * mut / P.prandtl_t;
    const double muT = mu + mut;
    const double div = du[0][0] + du[1][1] + du[2][2];
    double tau[3][3];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c)
        tau[a][c] = muT * (du[a][c] + du[c][a] - (a == c ? 2.0 / 3.0 * div : 0.0));
    double qh[3];
    for (int c = 0; c < 3; ++c) qh[c] = -kap * f.g[(9 + c) * N + n];
    const double uu[3] = {f.u[n], f.v[n], f.w[n]};
    const double e = q[4 * N + n], p = f.p[n];
    // E_a - V_a for a = x, y, z
    double EV[3][5];
    for (int c = 0; c < 3; ++c) {
      EV[c][0] = q[n] * uu[c];
      for (int r = 0; r < 3; ++r)
        EV[c][1 + r] = q[(1 + r) * N + n] * uu[c] + (r == c ? p : 0.0) - tau[r][c];
      EV[c][4] = (e + p) * uu[c] - (uu[0] * tau[0][c] + uu[1] * tau[1][c] + uu[2] * tau[2][c] - qh[c]);
    }
    for (int d = 0; d < 3; ++d)
      for (int v = 0; v < 5; ++v) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) acc += m[(3 * d + c) * N + n] * EV[c][v];
        f.F[(5 * d + v) * N + n] = acc;
      }
    // spectral radii lambda^d = |U^d| + a |grad xi_d|, U^d = J S^d . u
    for (int d = 0; d < 3; ++d) {
      const double* S = m + 3 * d * N;
      const double sx = S[n], sy = S[N + n], sz = S[2 * N + n];
      const double U = J * (sx * uu[0] + sy * uu[1] + sz * uu[2]);
      f.lam[d * N + n] = std::fabs(U) + f.a[n] * std::fabs(J) * std::sqrt(sx * sx + sy * sy + sz * sz);
    }
    // anisotropic scaling phi^d = 1 + sum_{d' != d} (lambda^d' / lambda^d)^alpha,
    // sigma^d = phi^d lambda^d / J
    for (int d = 0; d < 3; ++d) {
      const double ld = f.lam[d * N + n];
      double phi = 1.0;
      for (int e2 = 0; e2 < 3; ++e2)
        if (e2 != d) phi += std::pow(f.lam[e2 * N + n] / ld, P.tv_alpha);
      f.sig[d * N + n] = phi * ld / J;
    }
  }

  // pressure sensor along each direction
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b.n[2]; ++k)
    for (int j = 0; j < b.n[1]; ++j)
      for (int i = 0; i < b.n[0]; ++i) {
        const long n = b.at(i, j, k);
        for (int d = 0; d < 3; ++d) {
          const double pp = f.p[b.nb(i, j, k, d, +1)], pm = f.p[b.nb(i, j, k, d, -1)];
          f.nu[d * N + n] = std::fabs(pp - 2.0 * f.p[n] + pm) / (pp + 2.0 * f.p[n] + pm);
        }
      }
}

// Residual R = J (C - D):  C = sum_d delta_d F^d (centred), D = sum_d of the
// differences of the face dissipation fluxes d_{i+1/2} - d_{i-1/2}.
static void residual(const Block& b, const jzo_params& P, const double* m, const double* q,
                     double* r, Fields& f) {
  node_fields(b, P, m, q, f);
  const long N = b.N;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < b.n[2]; ++k)
    for (int j = 0; j < b.n[1]; ++j)
      for (int i = 0; i < b.n[0]; ++i) {
        const long n = b.at(i, j, k);
        if (!b.interior(i, j, k)) {  // boundary layers carry no residual
          for (int v = 0; v < 5; ++v) r[v * N + n] = 0.0;
          continue;
        }
        double C[5] = {0, 0, 0, 0, 0}, D[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d < 3; ++d) {
          const long np1 = b.nb(i, j, k, d, +1), nm1 = b.nb(i, j, k, d, -1);
          for (int v = 0; v < 5; ++v)
            C[v] += 0.5 * (f.F[(5 * d + v) * N + np1] - f.F[(5 * d + v) * N + nm1]);
          // faces i+1/2 (s = +1) and i-1/2 (s = -1) along d
          for (int s = -1; s <= 1; s += 2) {
            // the face lies between nodes L (left) and L+1
            const int off = (s > 0) ? 0 : -1;
            const long nL = b.nb(i, j, k, d, off), nR = b.nb(i, j, k, d, off + 1);
            const long nLL = b.nb(i, j, k, d, off - 1), nRR = b.nb(i, j, k, d, off + 2);
            const double eps2 = P.k2 * std::max(f.nu[d * N + nL], f.nu[d * N + nR]);
            const double eps4 = std::max(0.0, P.k4 - eps2);
            const double sg = 0.5 * (f.sig[d * N + nL] + f.sig[d * N + nR]);
            for (int v = 0; v < 5; ++v) {
              const double* Q = q + v * N;
              // third difference Q[i+2] - 3 Q[i+1] + 3 Q[i] - Q[i-1], differences
              // taken first so that a uniform field gives exactly zero
              const double d3 = (Q[nRR] - Q[nLL]) - 3.0 * (Q[nR] - Q[nL]);
              const double dface = sg * (eps2 * (Q[nR] - Q[nL]) - eps4 * d3);
              D[v] += s * dface;
            }
          }
        }
        const double J = m[9 * N + n];
        for (int v = 0; v < 5; ++v) r[v * N + n] = J * (C[v] - D[v]);
      }
}

static double cfl_max(const Block& b, const double* m, const double* q, const jzo_params& P) {
  // max over the interior nodes of lambda^xi + lambda^eta + lambda^zeta (inviscid)
  const long N = b.N;
  double mx = 0.0;
#pragma omp parallel for reduction(max : mx) schedule(static)
  for (int k = 0; k < b.n[2]; ++k)
    for (int j = 0; j < b.n[1]; ++j)
      for (int i = 0; i < b.n[0]; ++i) {
        if (!b.interior(i, j, k)) continue;
        const long n = b.at(i, j, k);
        const double rho = q[n];
        const double u = q[N + n] / rho, v = q[2 * N + n] / rho, w = q[3 * N + n] / rho;
        const double p = (P.gamma - 1.0) * (q[4 * N + n] - 0.5 * rho * (u * u + v * v + w * w));
        const double a = std::sqrt(P.gamma * p / rho);
        const double J = m[9 * N + n];
        double sum = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double sx = m[(3 * d) * N + n], sy = m[(3 * d + 1) * N + n], sz = m[(3 * d + 2) * N + n];
          sum += std::fabs(J * (sx * u + sy * v + sz * w)) + a * std::fabs(J) * std::sqrt(sx * sx + sy * sy + sz * sz);
        }
        mx = std::max(mx, sum);
      }
  return mx;
}

// Far-field state from Riemann invariants of the one-dimensional flow normal
// to the boundary (outward unit normal nh): the outgoing invariant
// R+ = u_n + 2a/(gamma-1) comes from the interior state qi, the incoming
// R- = u_n - 2a/(gamma-1) from the free stream; their half sum and difference
// give the normal velocity and sound speed at the boundary.  Entropy p/rho^gamma
// and the tangential velocity come from the upwind side (interior on outflow,
// free stream on inflow).  A supersonic normal flow takes every quantity
// from its upwind side.  Free stream: rho = 1, u = (mach_inf, 0, 0), p = 1/gamma.
static void farfield_state(const jzo_params& P, const double qi[5], const double nh[3], double qb[5]) {
  const double g = P.gamma;
  const double ri = qi[0];
  const double ui[3] = {qi[1] / ri, qi[2] / ri, qi[3] / ri};
  const double pi = (g - 1.0) * (qi[4] - 0.5 * ri * (ui[0] * ui[0] + ui[1] * ui[1] + ui[2] * ui[2]));
  const double ai = std::sqrt(g * pi / ri);
  const double re = 1.0, pe = 1.0 / g, ae = 1.0;
  const double ue[3] = {P.mach_inf, 0.0, 0.0};
  const double uni = ui[0] * nh[0] + ui[1] * nh[1] + ui[2] * nh[2];
  const double une = ue[0] * nh[0] + ue[1] * nh[1] + ue[2] * nh[2];
  double rb, ub[3], pb;
  if (uni >= ai) {  // supersonic outflow: everything from the interior
    rb = ri;
    pb = pi;
    for (int a = 0; a < 3; ++a) ub[a] = ui[a];
  } else if (uni <= -ai) {  // supersonic inflow: everything from the free stream
    rb = re;
    pb = pe;
    for (int a = 0; a < 3; ++a) ub[a] = ue[a];
  } else {
    const double rp = uni + 2.0 * ai / (g - 1.0);
    const double rm = une - 2.0 * ae / (g - 1.0);
    const double unb = 0.5 * (rp + rm);
    const double ab = 0.25 * (g - 1.0) * (rp - rm);
    const bool out = unb > 0.0;
    const double ent = out ? pi / std::pow(ri, g) : pe / std::pow(re, g);
    const double* ut = out ? ui : ue;
    const double unt = out ? uni : une;
    for (int a = 0; a < 3; ++a) ub[a] = ut[a] + (unb - unt) * nh[a];
    rb = std::pow(ab * ab / (g * ent), 1.0 / (g - 1.0));
    pb = rb * ab * ab / g;
  }
  qb[0] = rb;
  for (int a = 0; a < 3; ++a) qb[1 + a] = rb * ub[a];
  qb[4] = pb / (g - 1.0) + 0.5 * rb * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
}

// Boundary conditions on a state q after a stage (Sec. 3, boundary
// conditions): for each bounded direction in the order xi, eta, zeta, every
// node of its two boundary layers at each end is set from its face's rule --
// supersonic inflow holds the value the node has in q0 (the state given at
// the start of the step), far field applies farfield_state to the first
// interior node along the direction (index 2, or n-3) with the face's
// outward normal at the boundary node, and the centreline face of a
// cylindrical mesh (eta = 0 is the axis) extrapolates the conserved variables
// from the first advanced ring (j = 2) to the ring j = 1 and sets the axis
// nodes j = 0 of every azimuth k to their average over k of that ring, summed
// in the order k = 0, 1, ..., nk-1 (Sec. 3; the fixed order is the paper's
// reproducibility rule of Sec. 4.3).  A node in the layers of an inflow
// face is held at its inflow value whatever other faces it also belongs to;
// otherwise a node in the boundary layers of several directions keeps the
// value of the last of them.
static void apply_bc(const Block& b, const jzo_params& P, const double* m, double* q, const double* q0) {
  const long N = b.N;
  for (int d = 0; d < 3; ++d) {
    if (!b.bnd[d]) continue;
    for (int k = 0; k < b.n[2]; ++k)
      for (int j = 0; j < b.n[1]; ++j)
        for (int i = 0; i < b.n[0]; ++i) {
          int c[3] = {i, j, k};
          const bool lo = c[d] < 2, hi = c[d] > b.n[d] - 3;
          if (!lo && !hi) continue;
          const long n = b.at(i, j, k);
          bool held = false;  // in the layers of some inflow face
          for (int e = 0; e < 3; ++e) {
            if (!b.bnd[e]) continue;
            if ((c[e] < 2 && P.bc[2 * e] == 1) || (c[e] > b.n[e] - 3 && P.bc[2 * e + 1] == 1)) held = true;
          }
          if (held) {
            for (int v = 0; v < 5; ++v) q[v * N + n] = q0[v * N + n];
            continue;
          }
          const int type = P.bc[2 * d + (hi ? 1 : 0)];
          if (type == 3) {  // centreline
            double acc[5] = {0, 0, 0, 0, 0};
            if (c[1] == 1) {
              for (int v = 0; v < 5; ++v) acc[v] = q[v * N + b.at(c[0], 2, c[2])];
            } else {
              for (int kk = 0; kk < b.n[2]; ++kk)
                for (int v = 0; v < 5; ++v) acc[v] += q[v * N + b.at(c[0], 2, kk)];
              for (int v = 0; v < 5; ++v) acc[v] /= (double)b.n[2];
            }
            for (int v = 0; v < 5; ++v) q[v * N + n] = acc[v];
            continue;
          }
          c[d] = lo ? 2 : b.n[d] - 3;
          const long nr = b.at(c[0], c[1], c[2]);
          double qi[5], qb[5], nh[3];
          for (int v = 0; v < 5; ++v) qi[v] = q[v * N + nr];
          // outward normal: -grad(xi_d) on the low face, +grad(xi_d) on the high face
          const double J = m[9 * N + n];
          double len = 0.0;
          for (int a = 0; a < 3; ++a) {
            nh[a] = J * m[(3 * d + a) * N + n];
            len += nh[a] * nh[a];
          }
          len = std::sqrt(len);
          for (int a = 0; a < 3; ++a) nh[a] = (lo ? -nh[a] : nh[a]) / len;
          farfield_state(P, qi, nh, qb);
          for (int v = 0; v < 5; ++v) q[v * N + n] = qb[v];
        }
  }
}

static bool check(int ni, int nj, int nk, const jzo_params* p, const void* a, const void* b2) {
  if (!(ni >= 1 && nj >= 1 && nk >= 1 && p && a && b2 && p->n_stages >= 1 && p->n_stages <= 5)) return false;
  const int n[3] = {ni, nj, nk};
  for (int d = 0; d < 3; ++d) {
    const int lo = p->bc[2 * d], hi = p->bc[2 * d + 1];
    if (lo < 0 || lo > 3 || hi < 0 || hi > 3) return false;
    if ((lo == 0) != (hi == 0)) return false;   // periodic faces come in pairs
    if (lo != 0 && n[d] < 5) return false;      // two boundary layers at each end
  }
  // the centreline is the eta- face of a mesh periodic in zeta (azimuth)
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] == 3 && (f != 2 || p->bc[4] != 0)) return false;
  return true;
}

}  // namespace

extern "C" {

// R(Q) for the whole block (5 x N, SoA).
int jzo_residual(int ni, int nj, int nk, const jzo_params* P, const double* m, const double* q,
                 double* r) {
  if (!check(ni, nj, nk, P, m, q) || !r) return -1;
  Block b(ni, nj, nk, P->bc);
  Fields f(b.N);
  residual(b, *P, m, q, r, f);
  return 0;
}

// Diagnostic node fields of R(Q): mu, mu_t (N each), lambda (3 x N),
// sigma (3 x N), sensor nu (3 x N), gradients (12 x N).  Any pointer may be NULL.
int jzo_fields(int ni, int nj, int nk, const jzo_params* P, const double* m, const double* q,
               double* mu, double* mut, double* lam, double* sig, double* nu, double* grad) {
  if (!check(ni, nj, nk, P, m, q)) return -1;
  Block b(ni, nj, nk, P->bc);
  Fields f(b.N);
  node_fields(b, *P, m, q, f);
  const long N = b.N;
  if (mu) std::memcpy(mu, f.mu.data(), N * sizeof(double));
  if (mut) std::memcpy(mut, f.mut.data(), N * sizeof(double));
  if (lam) std::memcpy(lam, f.lam.data(), 3 * N * sizeof(double));
  if (sig) std::memcpy(sig, f.sig.data(), 3 * N * sizeof(double));
  if (nu) std::memcpy(nu, f.nu.data(), 3 * N * sizeof(double));
  if (grad) std::memcpy(grad, f.g.data(), 12 * N * sizeof(double));
  return 0;
}

// Global time step dt = cfl / max_nodes sum_d lambda^d (or dt_fixed).
int jzo_cfl_dt(int ni, int nj, int nk, const jzo_params* P, const double* m, const double* q,
               double* dt, double* lam_max) {
  if (!check(ni, nj, nk, P, m, q) || !dt) return -1;
  Block b(ni, nj, nk, P->bc);
  const double mx = cfl_max(b, m, q, *P);
  if (lam_max) *lam_max = mx;
  *dt = (P->dt_fixed > 0.0) ? P->dt_fixed : P->cfl / mx;
  return 0;
}

// One explicit multistage step, in place on q (5 x N):
//   Q(0) = Q^n;  Q(k) = Q(0) - alpha_k dt R(Q(k-1)), k = 1..n_stages;  Q^{n+1} = Q(last).
// dt_in > 0 forces the step size; otherwise it follows the CFL rule on Q^n.
// rms/linf (5 each, may be NULL) receive the norms of the first-stage R(Q^n).
int jzo_step(int ni, int nj, int nk, const jzo_params* P, const double* m, double* q, double dt_in,
             double* dt_used, double* rms, double* linf) {
  if (!check(ni, nj, nk, P, m, q)) return -1;
  Block b(ni, nj, nk, P->bc);
  const long N = b.N;
  double dt = dt_in;
  if (!(dt > 0.0)) {
    const double mx = cfl_max(b, m, q, *P);
    dt = (P->dt_fixed > 0.0) ? P->dt_fixed : P->cfl / mx;
  }
  if (dt_used) *dt_used = dt;
  std::vector<double> q0(q, q + 5 * N), qk(q, q + 5 * N), r(5 * N);
  Fields f(N);
  for (int s = 0; s < P->n_stages; ++s) {
    residual(b, *P, m, qk.data(), r.data(), f);  // zero on boundary layers
    if (s == 0) {
      // norms over the interior nodes (all nodes of a periodic block)
      const double nint = (double)b.n_interior();
      for (int v = 0; v < 5; ++v) {
        double ss = 0.0, mx = 0.0;
        for (long n = 0; n < N; ++n) {
          const double x = r[v * N + n];
          ss += x * x;
          mx = std::max(mx, std::fabs(x));
        }
        if (rms) rms[v] = std::sqrt(ss / nint);
        if (linf) linf[v] = mx;
      }
    }
    const double ad = P->rk_alpha[s] * dt;
    for (long n = 0; n < 5 * N; ++n) qk[n] = q0[n] - ad * r[n];
    apply_bc(b, *P, m, qk.data(), q0.data());
  }
  std::memcpy(q, qk.data(), 5 * N * sizeof(double));
  return 0;
}

// The boundary conditions alone, in place on q (5 x N): inflow layers take
// their values from q0, far-field layers are recomputed from q.
int jzo_apply_bc(int ni, int nj, int nk, const jzo_params* P, const double* m, double* q, const double* q0) {
  if (!check(ni, nj, nk, P, m, q) || !q0) return -1;
  Block b(ni, nj, nk, P->bc);
  apply_bc(b, *P, m, q, q0);
  return 0;
}

// Worker threads of the loops (for timing the oracle at a given core count):
// n > 0 sets them; returns the count the next loop will use.
int jzo_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

// nsteps steps; *t accumulates the simulated time.
int jzo_advance(int ni, int nj, int nk, const jzo_params* P, const double* m, double* q, int nsteps,
                double* t, double* rms, double* linf) {
  if (nsteps < 0) return -1;
  for (int s = 0; s < nsteps; ++s) {
    double dt = 0.0;
    const int rc = jzo_step(ni, nj, nk, P, m, q, 0.0, &dt, rms, linf);
    if (rc) return rc;
    if (t) *t += dt;
  }
  return 0;
}

}  // extern "C"
