// jz_api.hip -- C ABI of the jet-LES library (host side).  See include/jetles.h.
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jetles.h"
#include "jz_internal.h"

namespace jz {
hipError_t launch_stage_fp64(const StageArgs& a, const int* flag, int mode, int bx, int by, int nblocks,
                             hipStream_t st);
hipError_t launch_stage_fp32(const StageArgs& a, const int* flag, int kind, int bx, int by, int nblocks,
                             hipStream_t st);
bool stage_shape_supported(int bx, int by);
bool stage32_shape_supported(int bx, int by);
bool batch64_shape_supported(int bx, int by);
int stage_wg_per_cu_fp64(int bx, int by);
int stage_wg_per_cu_fp32(int bx, int by);
bool batch32_shape_supported(int bx, int by);
hipError_t launch_stage_batch_fp64(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                                   int bx, int by, hipStream_t st);
hipError_t launch_stage_batch_fp32(const BlockDesc* d, const int* off, BatchCtl* ctl, int stage, int ns, double alpha,
                                   int bx, int by, hipStream_t st);
hipError_t launch_finalize_batch(const BlockDesc* desc, BatchCtl* ctl, int slots, hipStream_t st);
hipError_t launch_met32_to_soa(const float* m32, const double* jac, double* dst, long long N, hipStream_t st);
hipError_t launch_stats_accumulate(const double* q, double* acc, long long N, double gamma, hipStream_t st);
hipError_t launch_stats_finalize(const double* acc, long long N, double inv_n, double* out, hipStream_t st);
hipError_t launch_stats_profile(const double* soa, long long N, int ni, int nj, int nk, int i, const int* bins,
                                int nbins, double* out, hipStream_t st);
hipError_t launch_bc(void* q, bool q_float, const double* q0, const void* met, const double* jac, bool met32,
                     const int n[3], const int bc[6], double gamma, double mach_inf, double* axis_mean,
                     const double* ref, hipStream_t st);
hipError_t launch_metrics_tl(const double* X, const double* period9, int ni, int nj, int nk, int bnd, void* m, double* jac,
                             bool met32, hipStream_t st);
hipError_t launch_check_met32(const float* m32, const double* jac, long long N, int axis_ni, int axis_nj, int* flag,
                              hipStream_t st);
hipError_t launch_soa_to_met32(const double* src, float* m32, double* jac, long long N, hipStream_t st);
hipError_t launch_soa_to_nodes(const double* src, double* dst, long long N, int C, hipStream_t st);
hipError_t launch_nodes_to_soa(const double* src, double* dst, long long N, int C, hipStream_t st);
hipError_t launch_check_metrics(const double* m, long long N, int axis_ni, int axis_nj, int* flag, hipStream_t st);
hipError_t launch_check_state(const double* q, long long N, double gm1, int* flag, hipStream_t st);
int lambda_max_blocks(long long N);
hipError_t launch_lambda_max(const double* q, const void* met, const double* jac, bool met32, long long N,
                             const int n[3], Interior in, double gamma, double* part, hipStream_t st);
hipError_t launch_finalize_dt(Clock* clk, const double* lam_part, int nb, StepCtl ctl, int* flag, hipStream_t st);
hipError_t launch_finalize_step(Clock* clk, const double* norm_part, const double* lam_part, int nb, StepCtl ctl,
                                int* flag, hipStream_t st);
hipError_t launch_reset_clock(Clock* clk, int* flag, hipStream_t st);
hipError_t launch_domain_dt(const DomainSub* sub, int P, StepCtl ctl, hipStream_t st);
hipError_t launch_domain_finalize(const DomainSub* sub, int P, StepCtl ctl, BatchCtl* work, double* part_red,
                                  hipStream_t st);
hipError_t launch_halo_jobs(const HaloJob* jobs, int njobs, bool is_float, int d, long long max_count,
                            hipStream_t st);
hipError_t launch_export_clock(const Clock* clk, const int* flag, double* out, hipStream_t st);
}  // namespace jz

using namespace jz;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(JZ_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Device workspace.  Q0 and every stage state are node-major (5 values per
// node).  "stage" is a scratch region of Np-rounded rows (Np = N rounded up to
// 32): its halves A and B (5 x Np doubles each) are the FP64 stage buffers
// Qa/Qb, and between steps it stages transposes, coordinates and metrics.
//   FP64:      Q0 | stage (10 Np doubles) | metrics (10 doubles per node)
//   FP32-flux: Q0 | stage (10 Np doubles; during a step its first 10 Np
//              floats are the float stage states Q32a, Q32b) | metrics
//              (9 floats per node) | J (1 double per node)
struct Layout {
  size_t q0, stage, q32a, q32b, met, jac, norm_part, lam_part, clock, flag, stats, axis, ref, total;
  long long np;
};

// bit d set when direction d has physical faces
int bounded_mask(const jz_params* p) {
  int m = 0;
  for (int d = 0; d < 3; ++d)
    if (p && p->bc[2 * d] != JZ_BC_PERIODIC) m |= 1 << d;
  return m;
}

// the nodes the residual advances (all of a periodic direction; a bounded one
// loses its two boundary layers at each end)
Interior interior_of(int ni, int nj, int nk, const jz_params* p) {
  Interior in;
  const int n[3] = {ni, nj, nk};
  in.bnd = bounded_mask(p);
  for (int d = 0; d < 3; ++d) {
    const bool b = (in.bnd >> d) & 1;
    in.lo[d] = b ? 2 : 0;
    in.hi[d] = b ? n[d] - 2 : n[d];
  }
  return in;
}

long long interior_count(const Interior& in) {
  return (long long)(in.hi[0] - in.lo[0]) * (in.hi[1] - in.lo[1]) * (in.hi[2] - in.lo[2]);
}

// `over`: the nodes to tile when they are not the parameters' own interior
// (the sub-blocks of a domain, whose ghost layers are not advanced)
void pick_tiling(int ni, int nj, int nk, const jz_params* p, Tiling* t, const Interior* over = nullptr) {
  const bool f32 = p && p->precision == JZ_FP32_FLUX;
  // defaults measured on the 512 x 256 x 256 workload: tile rows of 16 or 32
  // owned columns (whole 16-lane groups, so a row's LDS reads meet no bank
  // conflict); FP64 16 x 12 tiles in the compact form (256 threads, one
  // wave per SIMD, two workgroups per CU; 8 % ahead of 16 x 16 tiles with
  // partner waves), FP32-flux 32 x 16 tiles (720 threads, three waves per SIMD)
  t->bx = f32 ? 36 : 20;
  t->by = f32 ? 20 : 16;
  if (p && p->tile_i > 0 && p->tile_j > 0) {
    t->bx = p->tile_i + 4;
    t->by = p->tile_j + 4;
  }
  t->ti = t->bx - 4;
  t->tj = t->by - 4;
  // tiles and chunks cover the advanced nodes only
  const Interior in = over ? *over : interior_of(ni, nj, nk, p);
  const int ei = in.hi[0] - in.lo[0], ej = in.hi[1] - in.lo[1], ek = in.hi[2] - in.lo[2];
  t->tiles_i = (ei + t->ti - 1) / t->ti;
  t->tiles_j = (ej + t->tj - 1) / t->tj;
  int kc = (p && p->kchunk > 0) ? p->kchunk : 64;
  if (kc > ek) kc = ek;
  t->kchunk = kc;
  t->nchunks = (ek + kc - 1) / kc;
  t->nblocks = t->tiles_i * t->tiles_j * t->nchunks;
}

// Planes per chunk when the caller leaves it to the library.  Every workgroup
// marches kc + 2 planes (two warm-up planes), and the workgroups run in
// rounds of `slots` (workgroups resident on the whole device), so a launch
// costs about ceil(tiles * chunks / slots) * (kc + 2) plane steps.  The
// chunk length minimising that count fills the last round instead of leaving
// most CUs idle in it; ties go to the longer chunk (fewer halo re-reads).
// Chunks are at least 8 planes (the partial-sum arrays are sized for that).
int auto_kchunk(int tiles, int nk, long long slots) {
  if (nk <= 8 || slots < 1) return nk < 64 ? nk : 64;
  int best_kc = nk;
  long long best = -1;
  for (int c = 1; c <= (nk + 7) / 8; ++c) {
    const int kc = (nk + c - 1) / c;
    if (kc < 8) break;
    const long long chunks = (nk + kc - 1) / kc;
    const long long rounds = ((long long)tiles * chunks + slots - 1) / slots;
    const long long cost = rounds * (kc + 2);
    if (best < 0 || cost < best || (cost == best && kc > best_kc)) {
      best = cost;
      best_kc = kc;
    }
  }
  return best_kc;
}

// pick_tiling, then (kchunk left to the library) the chunk length for the
// current device's CU count and the shape's occupancy
void pick_tiling_for_device(int ni, int nj, int nk, const jz_params* p, Tiling* t, const Interior* over = nullptr) {
  pick_tiling(ni, nj, nk, p, t, over);
  if (p && p->kchunk > 0) return;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return;
  const int per_cu = (p && p->precision == JZ_FP32_FLUX) ? stage_wg_per_cu_fp32(t->bx, t->by)
                                                          : stage_wg_per_cu_fp64(t->bx, t->by);
  if (per_cu < 1 || ncu < 1) return;
  const Interior in = over ? *over : interior_of(ni, nj, nk, p);
  const int ek = in.hi[2] - in.lo[2];
  // The compact FP64 shape (16 x 12 tiles, two workgroups per CU) runs its
  // workgroups unsynchronised, so the rounds model does not hold for it;
  // chunks of 64 planes measured best on 512 x 256 x 256 (32: +2 %, 128: +6 %).
  // A block too small to give every resident workgroup slot a tile with
  // such chunks takes shorter ones, as many as fill the device.
  const bool compact = (!p || p->precision == JZ_FP64) && t->bx == 20 && t->by == 16;
  const long long slots = (long long)per_cu * ncu, tiles = (long long)t->tiles_i * t->tiles_j;
  int kc = 0;
  if (compact) {
    kc = ek < 64 ? ek : 64;
    if (tiles * ((ek + kc - 1) / kc) < slots) kc = auto_kchunk((int)tiles, ek, slots);
  } else {
    kc = auto_kchunk((int)tiles, ek, slots);
  }
  t->kchunk = kc;
  t->nchunks = (ek + kc - 1) / kc;
  t->nblocks = t->tiles_i * t->tiles_j * t->nchunks;
}

// Tiles of the finest supported tiling (interior 12 x 4 tiles with 8-plane
// chunks bounds every shape in either precision), so the partial-sum arrays
// never need to grow when the tiling changes.
int partial_capacity(int ni, int nj, int nk, const Tiling& t) {
  const int fine = ((ni + 11) / 12) * ((nj + 3) / 4) * ((nk + 7) / 8);
  return fine > t.nblocks ? fine : t.nblocks;
}

Layout layout_for(long long N, const Tiling& t, int prec, int cap, bool stats, int axis_ni, long long ref_nodes) {
  Layout L;
  std::memset(&L, 0, sizeof L);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.np = (N + 31) / 32 * 32;
  L.q0 = take(5 * N * sizeof(double));
  L.stage = take(10 * L.np * sizeof(double));
  if (prec == JZ_FP64) {
    L.met = take(10 * N * sizeof(double));
  } else {
    L.q32a = L.stage;
    L.q32b = L.stage + 5 * L.np * sizeof(float);
    L.met = take(9 * N * sizeof(float));
    L.jac = take(N * sizeof(double));
  }
  L.norm_part = take((size_t)cap * 10 * sizeof(double));
  const int lb = cap > lambda_max_blocks(N) ? cap : lambda_max_blocks(N);
  L.lam_part = take((size_t)lb * sizeof(double));
  L.clock = take(sizeof(Clock));
  L.flag = take(4 * sizeof(int));
  // time-averaged statistics: sums of u, u^2, p, p^2 per node (node-major)
  L.stats = stats ? take(4 * N * sizeof(double)) : 0;
  // centreline: the azimuthal mean of the five conserved variables at each
  // axial station (computed once per stage, read by every axis node)
  L.axis = axis_ni > 0 ? take((size_t)axis_ni * 5 * sizeof(double)) : 0;
  // FP32-flux with physical faces: the double states of the far-field
  // reference planes (see StageArgs::ref)
  L.ref = ref_nodes > 0 ? take((size_t)ref_nodes * 5 * sizeof(double)) : 0;
  L.total = off;
  return L;
}

// nodes of the FP32-flux far-field reference buffer (0: none needed)
long long ref_nodes_of(int ni, int nj, int nk, const jz_params* p) {
  if (!p || p->precision != JZ_FP32_FLUX || !bounded_mask(p)) return 0;
  const int n[3] = {ni, nj, nk};
  long long off[3];
  return ref_layout(n, bounded_mask(p), off);
}

bool params_ok(const jz_params* p, std::string* why) {
  if (!p) {
    *why = "params is NULL";
    return false;
  }
  if (!(p->gamma > 1.0) || !(p->prandtl > 0) || !(p->prandtl_t > 0) || !(p->sutherland_s > 0) || !(p->cs >= 0) ||
      !(p->k2 >= 0) || !(p->k4 >= 0) || !(p->tv_alpha >= 0) || !(p->cfl > 0) || !(p->dt_fixed >= 0) ||
      !(p->mach_j >= 0)) {
    *why = "a physical or numerical parameter is out of range";
    return false;
  }
  if (p->n_stages < 1 || p->n_stages > 5) {
    *why = "n_stages must be 1..5";
    return false;
  }
  if (p->precision != JZ_FP64 && p->precision != JZ_FP32_FLUX) {
    *why = "precision must be JZ_FP64 or JZ_FP32_FLUX";
    return false;
  }
  if ((p->tile_i > 0) != (p->tile_j > 0)) {
    *why = "tile_i and tile_j must both be set or both be 0";
    return false;
  }
  if (p->tile_i > 0 && p->precision == JZ_FP64 && !stage_shape_supported(p->tile_i + 4, p->tile_j + 4)) {
    *why = "unsupported FP64 tile shape (supported: 16x12, 16x16, 28x12, 60x4, 12x28, 28x4, 12x12, 32x8)";
    return false;
  }
  if (p->tile_i > 0 && p->precision == JZ_FP32_FLUX && !stage32_shape_supported(p->tile_i + 4, p->tile_j + 4)) {
    *why = "unsupported FP32-flux tile shape (supported: 28x12, 28x20, 12x12, 32x16)";
    return false;
  }
  if (p->kchunk < 0) {
    *why = "kchunk must be >= 0";
    return false;
  }
  if (p->stats_interval < 0) {
    *why = "stats_interval must be >= 0";
    return false;
  }
  for (int d = 0; d < 3; ++d) {
    const int lo = p->bc[2 * d], hi = p->bc[2 * d + 1];
    if (lo < JZ_BC_PERIODIC || lo > JZ_BC_AXIS || hi < JZ_BC_PERIODIC || hi > JZ_BC_AXIS) {
      *why = "bc values must be JZ_BC_PERIODIC, JZ_BC_INFLOW, JZ_BC_FARFIELD or JZ_BC_AXIS";
      return false;
    }
    if ((lo == JZ_BC_PERIODIC) != (hi == JZ_BC_PERIODIC)) {
      *why = "a direction is periodic at both faces or at neither";
      return false;
    }
  }
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] == JZ_BC_AXIS && (f != 2 || p->bc[4] != JZ_BC_PERIODIC)) {
      *why = "JZ_BC_AXIS is the eta- face of a mesh periodic in zeta";
      return false;
    }
  if (!std::isfinite(p->mach_inf)) {
    *why = "mach_inf must be finite";
    return false;
  }
  return true;
}

// sizes against the boundary layout: a bounded direction needs 5 nodes
bool dims_ok(int ni, int nj, int nk, const jz_params* p, std::string* why) {
  const int n[3] = {ni, nj, nk};
  for (int d = 0; d < 3; ++d)
    if ((bounded_mask(p) >> d & 1) && n[d] < 5) {
      *why = "a direction with physical faces needs at least 5 nodes";
      return false;
    }
  return true;
}

Phys make_phys(const jz_params& p) {
  Phys ph;
  ph.gamma = p.gamma;
  ph.gm1 = p.gamma - 1.0;
  const double mu_inf = (p.re_d > 0.0 && std::isfinite(p.re_d)) ? p.mach_j / p.re_d : 0.0;
  ph.mu_suth = mu_inf * (1.0 + p.sutherland_s);
  ph.suth_s = p.sutherland_s;
  ph.cs2 = p.cs * p.cs;
  const double cp = 1.0 / (p.gamma - 1.0);
  ph.kap_lam = cp / p.prandtl;
  ph.kap_turb = cp / p.prandtl_t;
  ph.k2 = p.k2;
  ph.k4 = p.k4;
  ph.tv_alpha = p.tv_alpha;
  ph.alpha_half = (p.tv_alpha == 0.5) ? 1 : 0;
  ph.pad = 0;
  return ph;
}

}  // namespace

struct jz_solver {
  int ni, nj, nk;
  long long N;
  jz_params p;
  Phys ph;
  Tiling tl;
  Interior in;      // nodes the residual advances
  int cap;          // tiles the partial-sum arrays can hold
  Layout L;
  hipStream_t stream;
  char* ws;
  bool owns_ws;
  int device;
  bool grid_set, state_set, dt_valid;
  int prec;
  double* q0;
  double* qa;       // stage half A (FP64 stage buffer, transposes)
  double* qb;       // stage half B
  float* q32a;      // FP32-flux stage states
  float* q32b;
  void* met;        // double x 10 (FP64) or float x 9 (FP32-flux) per node
  double* jac;      // FP32-flux: J per node
  double* norm_part;
  double* lam_part;
  Clock* clock;
  int* flag;
  double* stats;          // sums of u, u^2, p, p^2 per node, or NULL
  double* axis_mean;      // centreline: azimuthal means per axial station, or NULL
  double* ref;            // FP32-flux far-field reference states, or NULL
  long long stat_samples; // samples in the sums
  long long stat_steps;   // steps since the last reset (samples every stats_interval)
  // timing: events recorded around stage launches (ev), and created ones
  // not in use (ev_free), filled by jz_set_timing so that jz_advance creates
  // none while it issues work
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
  std::vector<double> ev_bytes;
  double stage_ms_acc;
  long long stage_launches_acc;
  double stage_bytes_acc;
};

namespace {

// Shape, parameters, tiling and workspace layout of a solver (no device work).
void setup_shape(jz_solver* s, int ni, int nj, int nk, const jz_params* p) {
  s->ni = ni;
  s->nj = nj;
  s->nk = nk;
  s->N = (long long)ni * nj * nk;
  s->p = *p;
  s->ph = make_phys(*p);
  pick_tiling_for_device(ni, nj, nk, p, &s->tl);
  s->in = interior_of(ni, nj, nk, p);
  s->prec = p->precision;
  s->cap = partial_capacity(ni, nj, nk, s->tl);
  s->L = layout_for(s->N, s->tl, s->prec, s->cap, p->stats_interval > 0, p->bc[2] == JZ_BC_AXIS ? ni : 0,
                    ref_nodes_of(ni, nj, nk, p));
  s->timing = false;
  s->stage_ms_acc = 0;
  s->stage_launches_acc = 0;
  s->stage_bytes_acc = 0;
}

// Pointers of every array into the workspace s->ws (layout s->L).
void bind_workspace(jz_solver* s) {
  s->q0 = (double*)(s->ws + s->L.q0);
  s->qa = (double*)(s->ws + s->L.stage);
  s->qb = s->qa + 5 * s->L.np;
  s->q32a = s->prec == JZ_FP32_FLUX ? (float*)(s->ws + s->L.q32a) : nullptr;
  s->q32b = s->prec == JZ_FP32_FLUX ? (float*)(s->ws + s->L.q32b) : nullptr;  // both inside the scratch region
  s->met = (void*)(s->ws + s->L.met);
  s->jac = s->prec == JZ_FP32_FLUX ? (double*)(s->ws + s->L.jac) : nullptr;
  s->norm_part = (double*)(s->ws + s->L.norm_part);
  s->lam_part = (double*)(s->ws + s->L.lam_part);
  s->clock = (Clock*)(s->ws + s->L.clock);
  s->flag = (int*)(s->ws + s->L.flag);
  s->stats = s->L.stats ? (double*)(s->ws + s->L.stats) : nullptr;
  s->axis_mean = s->L.axis ? (double*)(s->ws + s->L.axis) : nullptr;
  s->ref = s->L.ref ? (double*)(s->ws + s->L.ref) : nullptr;
  s->stat_samples = 0;
  s->stat_steps = 0;
  s->grid_set = s->state_set = s->dt_valid = false;
}

}  // namespace

extern "C" {

int jz_params_default(jz_params* p) {
  if (!p) return fail(JZ_EINVAL, "jz_params_default: NULL");
  std::memset(p, 0, sizeof *p);
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
  p->precision = JZ_FP64;
  return JZ_OK;
}

size_t jz_workspace_bytes(int ni, int nj, int nk, const jz_params* p) {
  if (ni < 1 || nj < 1 || nk < 1) return 0;
  std::string why;
  jz_params d;
  if (!p) {
    jz_params_default(&d);
    p = &d;
  }
  if (!params_ok(p, &why) || !dims_ok(ni, nj, nk, p, &why)) return 0;
  Tiling t;
  pick_tiling(ni, nj, nk, p, &t);
  return layout_for((long long)ni * nj * nk, t, p->precision, partial_capacity(ni, nj, nk, t), p->stats_interval > 0,
                    p->bc[2] == JZ_BC_AXIS ? ni : 0, ref_nodes_of(ni, nj, nk, p))
      .total;
}

int jz_create(int ni, int nj, int nk, const jz_params* p, void* dev_workspace, size_t ws_bytes, void* hip_stream,
              jz_solver** out) {
  if (!out) return fail(JZ_EINVAL, "jz_create: out is NULL");
  *out = nullptr;
  if (ni < 1 || nj < 1 || nk < 1) return fail(JZ_EINVAL, "jz_create: sizes must be >= 1 (got %d %d %d)", ni, nj, nk);
  if ((long long)ni * nj > (1LL << 30) || (long long)ni * nj * nk > (1LL << 36))
    return fail(JZ_EINVAL, "jz_create: block too large");
  std::string why;
  if (!params_ok(p, &why) || !dims_ok(ni, nj, nk, p, &why)) return fail(JZ_EINVAL, "jz_create: %s", why.c_str());
  jz_solver* s = new jz_solver();
  setup_shape(s, ni, nj, nk, p);
  s->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return fail(JZ_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  if (dev_workspace) {
    if (ws_bytes < s->L.total) {
      delete s;
      return fail(JZ_EINVAL, "jz_create: workspace of %zu bytes < %zu needed", ws_bytes, s->L.total);
    }
    if (((uintptr_t)dev_workspace) % kAlign) {
      delete s;
      return fail(JZ_EINVAL, "jz_create: workspace must be %zu-byte aligned", kAlign);
    }
    s->ws = (char*)dev_workspace;
    s->owns_ws = false;
  } else {
    void* ptr = nullptr;
    e = hipMalloc(&ptr, s->L.total);
    if (e != hipSuccess) {
      delete s;
      return fail(JZ_ENOMEM, "hipMalloc(%zu): %s", s->L.total, hipGetErrorString(e));
    }
    s->ws = (char*)ptr;
    s->owns_ws = true;
  }
  bind_workspace(s);
  Clock c0;
  std::memset(&c0, 0, sizeof c0);
  int z[4] = {0, 0, 0, 0};
  e = hipMemcpyAsync(s->clock, &c0, sizeof c0, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->flag, z, sizeof z, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && s->stats) e = hipMemsetAsync(s->stats, 0, 4 * s->N * sizeof(double), s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    if (s->owns_ws) (void)hipFree(s->ws);
    delete s;
    return fail(JZ_EHIP, "jz_create: %s", hipGetErrorString(e));
  }
  *out = s;
  return JZ_OK;
}

static int read_flag(jz_solver* s, int* f) {
  HIP_TRY(hipMemcpyAsync(f, s->flag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return JZ_OK;
}

static int clear_flag(jz_solver* s) {
  const int z = 0;
  HIP_TRY(hipMemcpyAsync(s->flag, &z, sizeof z, hipMemcpyHostToDevice, s->stream));
  return JZ_OK;
}

// Validate the installed metric set (J > 0 and every value finite).
static int validate_metrics(jz_solver* s, const char* who) {
  int rc = clear_flag(s);
  if (rc) return rc;
  // the centreline of a cylindrical mesh (j = 0) carries no metrics
  const int axis_nj = s->p.bc[2] == JZ_BC_AXIS ? s->nj : 0;
  if (s->prec == JZ_FP64)
    HIP_TRY(launch_check_metrics((const double*)s->met, s->N, s->ni, axis_nj, s->flag, s->stream));
  else
    HIP_TRY(launch_check_met32((const float*)s->met, s->jac, s->N, s->ni, axis_nj, s->flag, s->stream));
  int f = 0;
  rc = read_flag(s, &f);
  if (rc) return rc;
  if (f) {
    s->grid_set = false;
    clear_flag(s);
    HIP_TRY(hipStreamSynchronize(s->stream));
    return fail(JZ_EINVAL, "%s: metric set has %s", who, (f & 1) ? "non-finite values" : "non-positive J");
  }
  s->grid_set = true;
  s->dt_valid = false;
  return JZ_OK;
}

int jz_set_grid_coords(jz_solver* s, const double* x, const double* y, const double* z, const double* period) {
  if (!s || !x || !y || !z || !period) return fail(JZ_EINVAL, "jz_set_grid_coords: NULL argument");
  const size_t bytes = s->N * sizeof(double);
  // coordinates are staged in the scratch region; the metric kernel writes
  // the stored layout directly (FP64 metrics, or float metrics + double J)
  double* X = s->qa;
  HIP_TRY(hipMemcpyAsync(X, x, bytes, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(X + s->N, y, bytes, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipMemcpyAsync(X + 2 * s->N, z, bytes, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(launch_metrics_tl(X, period, s->ni, s->nj, s->nk, s->in.bnd, s->met, s->jac, s->prec == JZ_FP32_FLUX,
                            s->stream));
  return validate_metrics(s, "jz_set_grid_coords");
}

int jz_set_grid_metrics(jz_solver* s, const double* m, int on_device) {
  if (!s || !m) return fail(JZ_EINVAL, "jz_set_grid_metrics: NULL argument");
  // stage the 10 x N array, then convert it to the stored layout
  HIP_TRY(hipMemcpyAsync(s->qa, m, 10 * s->N * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
  if (s->prec == JZ_FP64)
    HIP_TRY(launch_soa_to_nodes(s->qa, (double*)s->met, s->N, 10, s->stream));
  else
    HIP_TRY(launch_soa_to_met32(s->qa, (float*)s->met, s->jac, s->N, s->stream));
  return validate_metrics(s, "jz_set_grid_metrics");
}

int jz_get_grid_metrics(jz_solver* s, double* m, int on_device) {
  if (!s || !m) return fail(JZ_EINVAL, "jz_get_grid_metrics: NULL argument");
  if (!s->grid_set) return fail(JZ_ESTATE, "jz_get_grid_metrics: no grid set");
  if (s->prec == JZ_FP64) {
    HIP_TRY(launch_nodes_to_soa((const double*)s->met, s->qa, s->N, 10, s->stream));
  } else {
    HIP_TRY(launch_met32_to_soa((const float*)s->met, s->jac, s->qa, s->N, s->stream));
  }
  HIP_TRY(hipMemcpyAsync(m, s->qa, 10 * s->N * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return JZ_OK;
}

int jz_set_state(jz_solver* s, const double* q, int on_device) {
  if (!s || !q) return fail(JZ_EINVAL, "jz_set_state: NULL argument");
  // validate a node-major copy in Qa first so that a bad state leaves Q untouched
  HIP_TRY(hipMemcpyAsync(s->qb, q, 5 * s->N * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
  HIP_TRY(launch_soa_to_nodes(s->qb, s->qa, s->N, 5, s->stream));
  int rc = clear_flag(s);
  if (rc) return rc;
  HIP_TRY(launch_check_state(s->qa, s->N, s->ph.gm1, s->flag, s->stream));
  int f = 0;
  rc = read_flag(s, &f);
  if (rc) return rc;
  if (f) {
    clear_flag(s);
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (f & 1) return fail(JZ_ENONFINITE, "jz_set_state: state holds NaN/Inf");
    return fail(JZ_EINVAL, "jz_set_state: rho or p not positive somewhere");
  }
  HIP_TRY(hipMemcpyAsync(s->q0, s->qa, 5 * s->N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->state_set = true;
  s->dt_valid = false;
  return JZ_OK;
}

static StageArgs stage_args(jz_solver* s, const void* qin, void* qout, double alpha) {
  StageArgs a;
  a.qin = qin;
  a.q0 = s->q0;
  a.qout = qout;
  a.met = s->met;
  a.jac = s->jac;
  a.clock = s->clock;
  a.norm_part = s->norm_part;
  a.lam_part = s->lam_part;
  a.alpha = alpha;
  a.N = s->N;
  a.ni = s->ni;
  a.nj = s->nj;
  a.nk = s->nk;
  a.tiles_i = s->tl.tiles_i;
  a.tiles_j = s->tl.tiles_j;
  a.kchunk = s->tl.kchunk;
  a.nchunks = s->tl.nchunks;
  a.in = s->in;
  a.ph = s->ph;
  a.ref = nullptr;
  const int n[3] = {s->ni, s->nj, s->nk};
  ref_layout(n, s->in.bnd, a.ref_off);
  return a;
}

static StepCtl step_ctl(jz_solver* s) {
  StepCtl c;
  c.cfl = s->p.cfl;
  c.dt_fixed = s->p.dt_fixed;
  c.inv_n = 1.0 / (double)interior_count(s->in);
  return c;
}

static int ensure_dt(jz_solver* s) {
  if (s->dt_valid) return JZ_OK;
  const int n[3] = {s->ni, s->nj, s->nk};
  HIP_TRY(launch_lambda_max(s->q0, s->met, s->jac, s->prec == JZ_FP32_FLUX, s->N, n, s->in, s->p.gamma,
                            s->lam_part, s->stream));
  HIP_TRY(launch_finalize_dt(s->clock, s->lam_part, lambda_max_blocks(s->N), step_ctl(s), s->flag, s->stream));
  s->dt_valid = true;
  return JZ_OK;
}

// algorithmic HBM bytes of one stage launch: every array read or written once
static double stage_bytes(jz_solver* s, int stage) {
  const double n = (double)interior_count(s->in);
  const int ns = s->p.n_stages;
  if (s->prec == JZ_FP64) {
    if (stage == 0) return n * (40.0 + 80.0 + 40.0);  // Q^n (which is also Q0), metrics, Q(1)
    return n * (40.0 + 40.0 + 80.0 + 40.0);           // Q(k-1), Q0, metrics, Q(k)
  }
  const double met = 36.0 + 8.0;                      // 9 float metrics + double J
  const double in = stage == 0 ? 40.0 : 20.0;         // double Q^n, else float Q(k-1)
  const double q0 = stage == 0 ? 0.0 : 40.0;          // Q0 (stage 0 reads it as its stencil)
  const double out = stage == ns - 1 ? 40.0 : 20.0;   // double Q^{n+1}, else float Q(k)
  return n * (in + q0 + met + out);
}

// one stage launch in the solver's precision form; kind as in launch_stage_fp32
static hipError_t launch_stage(jz_solver* s, const StageArgs& a, int k, int ns, bool residual_only) {
  if (s->prec == JZ_FP64) {
    int mode = residual_only ? 4 : ((k == 0 ? 1 : 0) | (k == ns - 1 ? 2 : 0));
    return launch_stage_fp64(a, s->flag, mode, s->tl.bx, s->tl.by, s->tl.nblocks, s->stream);
  }
  int kind;
  if (residual_only)
    kind = 4;
  else if (ns == 1)
    kind = 3;
  else if (k == 0)
    kind = 0;
  else if (k == ns - 1)
    kind = 2;
  else
    kind = 1;
  return launch_stage_fp32(a, s->flag, kind, s->tl.bx, s->tl.by, s->tl.nblocks, s->stream);
}

// Event pairs for the stage timing come from a pool that jz_set_timing fills
// (kEventPool pairs); only a run of more launches than that creates events
// while work is issued.
constexpr int kEventPool = 640;

static int fill_event_pool(jz_solver* s, int pairs) {
  while ((int)s->ev_free.size() < pairs) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(JZ_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    s->ev_free.emplace_back(e0, e1);
  }
  return JZ_OK;
}

static int take_event_pair(jz_solver* s, hipEvent_t* e0, hipEvent_t* e1) {
  if (s->ev_free.empty()) {
    int rc = fill_event_pool(s, 1);
    if (rc) return rc;
  }
  *e0 = s->ev_free.back().first;
  *e1 = s->ev_free.back().second;
  s->ev_free.pop_back();
  return JZ_OK;
}

static void destroy_events(std::vector<std::pair<hipEvent_t, hipEvent_t>>& v) {
  for (auto& pr : v) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  v.clear();
}

// The steps of jz_advance on a solver whose grid and state are set: every
// launch on s->stream, no allocation, no synchronisation.
static int advance_steps(jz_solver* s, int nsteps) {
  int rc = ensure_dt(s);
  if (rc) return rc;
  const int ns = s->p.n_stages;
  for (int step = 0; step < nsteps; ++step) {
    // buffer rotation: Q0 -> A -> B -> A -> B -> Q0 (last stage in place:
    // Q(0) is read only at the node being written).  A and B are double
    // (FP64) or float (FP32-flux) stage states.
    const void* in = s->q0;
    void* bufA = s->prec == JZ_FP64 ? (void*)s->qa : (void*)s->q32a;
    void* bufB = s->prec == JZ_FP64 ? (void*)s->qb : (void*)s->q32b;
    for (int k = 0; k < ns; ++k) {
      const bool last = (k == ns - 1);
      // A single stage reads its stencil from Q(0): it writes the double
      // stage buffer A, which is then copied into Q(0), so that no workgroup
      // overwrites nodes another one still reads as halo.
      void* out = (ns == 1) ? (void*)s->qa : last ? (void*)s->q0 : ((k % 2 == 0) ? bufA : bufB);
      StageArgs a = stage_args(s, in, out, s->p.rk_alpha[k]);
      // a float stage state keeps the double states of its far-field reference planes
      const bool float_out = s->prec == JZ_FP32_FLUX && !last && ns > 1;
      if (float_out) a.ref = s->ref;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (s->timing) {
        int rc_ev = take_event_pair(s, &e0, &e1);
        if (rc_ev) return rc_ev;
        HIP_TRY(hipEventRecord(e0, s->stream));
      }
      HIP_TRY(launch_stage(s, a, k, ns, false));
      // the events bracket the stage kernel alone
      if (s->timing) {
        HIP_TRY(hipEventRecord(e1, s->stream));
        s->ev.emplace_back(e0, e1);
        s->ev_bytes.push_back(stage_bytes(s, k));
      }
      if (s->in.bnd) {
        const int n[3] = {s->ni, s->nj, s->nk};
        HIP_TRY(launch_bc(out, float_out, s->q0, s->met, s->jac, s->prec == JZ_FP32_FLUX, n, s->p.bc, s->p.gamma,
                          s->p.mach_inf, s->axis_mean, float_out ? s->ref : nullptr, s->stream));
      }
      if (ns == 1)
        HIP_TRY(hipMemcpyAsync(s->q0, s->qa, 5 * s->N * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
      in = out;
    }
    HIP_TRY(launch_finalize_step(s->clock, s->norm_part, s->lam_part, s->tl.nblocks, step_ctl(s), s->flag,
                                 s->stream));
    if (s->stats && ++s->stat_steps % s->p.stats_interval == 0) {
      HIP_TRY(launch_stats_accumulate(s->q0, s->stats, s->N, s->p.gamma, s->stream));
      ++s->stat_samples;
    }
  }
  return JZ_OK;
}

int jz_advance(jz_solver* s, int nsteps) {
  if (!s) return fail(JZ_EINVAL, "jz_advance: NULL solver");
  if (nsteps < 0) return fail(JZ_EINVAL, "jz_advance: nsteps < 0");
  if (!s->grid_set || !s->state_set) return fail(JZ_ESTATE, "jz_advance: grid and state must be set first");
  return advance_steps(s, nsteps);
}

static int check_health(jz_solver* s) {
  int f = 0;
  int rc = read_flag(s, &f);
  if (rc) return rc;
  if (f) return fail(JZ_ENONFINITE, "a step produced NaN/Inf norms or a non-positive dt");
  return JZ_OK;
}

int jz_get_state(jz_solver* s, double* q, int on_device) {
  if (!s || !q) return fail(JZ_EINVAL, "jz_get_state: NULL argument");
  if (!s->state_set) return fail(JZ_ESTATE, "jz_get_state: no state set");
  HIP_TRY(launch_nodes_to_soa(s->q0, s->qa, s->N, 5, s->stream));
  HIP_TRY(hipMemcpyAsync(q, s->qa, 5 * s->N * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  return check_health(s);
}

int jz_get_residual_norms(jz_solver* s, double rms[5], double linf[5]) {
  if (!s || !rms || !linf) return fail(JZ_EINVAL, "jz_get_residual_norms: NULL argument");
  Clock c;
  HIP_TRY(hipMemcpyAsync(&c, s->clock, sizeof c, hipMemcpyDeviceToHost, s->stream));
  int rc = check_health(s);
  for (int v = 0; v < 5; ++v) {
    rms[v] = c.rms[v];
    linf[v] = c.linf[v];
  }
  return rc;
}

int jz_get_clock(jz_solver* s, double* t, double* next_dt, long long* steps) {
  if (!s) return fail(JZ_EINVAL, "jz_get_clock: NULL solver");
  if (s->grid_set && s->state_set) {
    int rc = ensure_dt(s);
    if (rc) return rc;
  }
  Clock c;
  HIP_TRY(hipMemcpyAsync(&c, s->clock, sizeof c, hipMemcpyDeviceToHost, s->stream));
  int rc = check_health(s);
  if (t) *t = c.t;
  if (next_dt) *next_dt = c.dt;
  if (steps) *steps = c.steps;
  return rc;
}

int jz_set_clock(jz_solver* s, double t, long long steps) {
  if (!s) return fail(JZ_EINVAL, "jz_set_clock: NULL solver");
  Clock c;
  HIP_TRY(hipMemcpyAsync(&c, s->clock, sizeof c, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  c.t = t;
  c.steps = steps;
  HIP_TRY(hipMemcpyAsync(s->clock, &c, sizeof c, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return JZ_OK;
}

int jz_eval_residual(jz_solver* s, double* r, int on_device) {
  if (!s || !r) return fail(JZ_EINVAL, "jz_eval_residual: NULL argument");
  if (!s->grid_set || !s->state_set) return fail(JZ_ESTATE, "jz_eval_residual: grid and state must be set first");
  StageArgs a = stage_args(s, s->q0, s->qa, 0.0);
  if (s->in.bnd) HIP_TRY(hipMemsetAsync(s->qa, 0, 5 * s->N * sizeof(double), s->stream));  // boundary layers: R = 0
  HIP_TRY(launch_stage(s, a, 0, s->p.n_stages, true));
  HIP_TRY(launch_nodes_to_soa(s->qa, s->qb, s->N, 5, s->stream));
  HIP_TRY(hipMemcpyAsync(r, s->qb, 5 * s->N * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  return check_health(s);
}

int jz_eval_dt(jz_solver* s, double* dt, double* lambda_max) {
  if (!s || !dt) return fail(JZ_EINVAL, "jz_eval_dt: NULL argument");
  if (!s->grid_set || !s->state_set) return fail(JZ_ESTATE, "jz_eval_dt: grid and state must be set first");
  s->dt_valid = false;
  int rc = ensure_dt(s);
  if (rc) return rc;
  Clock c;
  HIP_TRY(hipMemcpyAsync(&c, s->clock, sizeof c, hipMemcpyDeviceToHost, s->stream));
  rc = check_health(s);
  *dt = c.dt;
  if (lambda_max) *lambda_max = c.lam_max;
  return rc;
}

int jz_stats_reset(jz_solver* s) {
  if (!s) return fail(JZ_EINVAL, "jz_stats_reset: NULL solver");
  if (!s->stats) return fail(JZ_ESTATE, "jz_stats_reset: statistics were not enabled (stats_interval = 0)");
  HIP_TRY(hipMemsetAsync(s->stats, 0, 4 * s->N * sizeof(double), s->stream));
  s->stat_samples = 0;
  s->stat_steps = 0;
  return JZ_OK;
}

int jz_stats_sample(jz_solver* s) {
  if (!s) return fail(JZ_EINVAL, "jz_stats_sample: NULL solver");
  if (!s->stats) return fail(JZ_ESTATE, "jz_stats_sample: statistics were not enabled (stats_interval = 0)");
  if (!s->state_set) return fail(JZ_ESTATE, "jz_stats_sample: no state set");
  HIP_TRY(launch_stats_accumulate(s->q0, s->stats, s->N, s->p.gamma, s->stream));
  ++s->stat_samples;
  return JZ_OK;
}

int jz_get_stats(jz_solver* s, double* mean_u, double* rms_u, double* mean_p, double* rms_p, long long* nsamples,
                 int on_device) {
  if (!s) return fail(JZ_EINVAL, "jz_get_stats: NULL solver");
  if (!s->stats) return fail(JZ_ESTATE, "jz_get_stats: statistics were not enabled (stats_interval = 0)");
  if (nsamples) *nsamples = s->stat_samples;
  if (s->stat_samples == 0) return fail(JZ_ESTATE, "jz_get_stats: no samples yet");
  HIP_TRY(launch_stats_finalize(s->stats, s->N, 1.0 / (double)s->stat_samples, s->qa, s->stream));
  double* outs[4] = {mean_u, rms_u, mean_p, rms_p};
  for (int f = 0; f < 4; ++f)
    if (outs[f])
      HIP_TRY(hipMemcpyAsync(outs[f], s->qa + f * s->N, s->N * sizeof(double),
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return JZ_OK;
}

int jz_stats_profile(jz_solver* s, int i, const int* bins, int nbins, double* mean_u, double* rms_u,
                     double* mean_p, double* rms_p, long long* counts) {
  if (!s || !bins) return fail(JZ_EINVAL, "jz_stats_profile: NULL argument");
  if (i < 0 || i >= s->ni || nbins < 1) return fail(JZ_EINVAL, "jz_stats_profile: i or nbins out of range");
  if (!s->stats) return fail(JZ_ESTATE, "jz_stats_profile: statistics were not enabled (stats_interval = 0)");
  if (s->stat_samples == 0) return fail(JZ_ESTATE, "jz_stats_profile: no samples yet");
  const long long plane = (long long)s->nj * s->nk;
  for (long long t = 0; t < plane; ++t)
    if (bins[t] < -1 || bins[t] >= nbins) return fail(JZ_EINVAL, "jz_stats_profile: bin index out of range");
  if (4 * s->N + (long long)nbins * 5 + (plane + 1) / 2 + 1 > 10 * s->L.np)
    return fail(JZ_EINVAL, "jz_stats_profile: too many bins for the scratch region");
  // scratch: node statistics (4 x N), bin results (5 x nbins), bin indices
  double* soa = s->qa;
  double* res = soa + 4 * s->N;
  int* dbins = (int*)(res + 5 * (long long)nbins);
  HIP_TRY(launch_stats_finalize(s->stats, s->N, 1.0 / (double)s->stat_samples, soa, s->stream));
  HIP_TRY(hipMemcpyAsync(dbins, bins, plane * sizeof(int), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(launch_stats_profile(soa, s->N, s->ni, s->nj, s->nk, i, dbins, nbins, res, s->stream));
  std::vector<double> h(5 * (size_t)nbins);
  HIP_TRY(hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int b = 0; b < nbins; ++b) {
    if (mean_u) mean_u[b] = h[5 * b + 0];
    if (rms_u) rms_u[b] = h[5 * b + 1];
    if (mean_p) mean_p[b] = h[5 * b + 2];
    if (rms_p) rms_p[b] = h[5 * b + 3];
    if (counts) counts[b] = (long long)h[5 * b + 4];
  }
  return JZ_OK;
}

int jz_set_timing(jz_solver* s, int enable) {
  if (!s) return fail(JZ_EINVAL, "jz_set_timing: NULL solver");
  HIP_TRY(hipStreamSynchronize(s->stream));
  // recorded events go back to the pool
  s->ev_free.insert(s->ev_free.end(), s->ev.begin(), s->ev.end());
  s->ev.clear();
  s->ev_bytes.clear();
  s->stage_ms_acc = 0;
  s->stage_launches_acc = 0;
  s->stage_bytes_acc = 0;
  s->timing = enable != 0;
  if (s->timing) return fill_event_pool(s, kEventPool);
  destroy_events(s->ev_free);
  return JZ_OK;
}

int jz_get_timing(jz_solver* s, double* stage_ms, long long* stage_launches, double* stage_bytes_out) {
  if (!s) return fail(JZ_EINVAL, "jz_get_timing: NULL solver");
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (size_t i = 0; i < s->ev.size(); ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, s->ev[i].first, s->ev[i].second));
    s->stage_ms_acc += ms;
    s->stage_launches_acc += 1;
    s->stage_bytes_acc += s->ev_bytes[i];
  }
  s->ev_free.insert(s->ev_free.end(), s->ev.begin(), s->ev.end());
  s->ev.clear();
  s->ev_bytes.clear();
  if (stage_ms) *stage_ms = s->stage_ms_acc;
  if (stage_launches) *stage_launches = s->stage_launches_acc;
  if (stage_bytes_out) *stage_bytes_out = s->stage_bytes_acc;
  return JZ_OK;
}

int jz_set_tiling(jz_solver* s, int tile_i, int tile_j, int kchunk) {
  if (!s) return fail(JZ_EINVAL, "jz_set_tiling: NULL solver");
  jz_params p = s->p;
  p.tile_i = tile_i;
  p.tile_j = tile_j;
  p.kchunk = kchunk;
  std::string why;
  if (!params_ok(&p, &why)) return fail(JZ_EINVAL, "jz_set_tiling: %s", why.c_str());
  Tiling t;
  pick_tiling_for_device(s->ni, s->nj, s->nk, &p, &t);
  if (t.nblocks > s->cap) return fail(JZ_EINVAL, "jz_set_tiling: %d tiles exceed the %d the workspace holds", t.nblocks, s->cap);
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->p = p;
  s->tl = t;
  return JZ_OK;
}

int jz_get_occupancy(jz_solver* s, int* wg_per_cu, int* cus) {
  if (!s) return fail(JZ_EINVAL, "jz_get_occupancy: NULL solver");
  int ncu = 0;
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device));
  const int per = s->prec == JZ_FP32_FLUX ? stage_wg_per_cu_fp32(s->tl.bx, s->tl.by)
                                           : stage_wg_per_cu_fp64(s->tl.bx, s->tl.by);
  if (wg_per_cu) *wg_per_cu = per;
  if (cus) *cus = ncu;
  return JZ_OK;
}

int jz_get_tiling(jz_solver* s, int* tile_i, int* tile_j, int* kchunk) {
  if (!s) return fail(JZ_EINVAL, "jz_get_tiling: NULL solver");
  if (tile_i) *tile_i = s->tl.ti;
  if (tile_j) *tile_j = s->tl.tj;
  if (kchunk) *kchunk = s->tl.kchunk;
  return JZ_OK;
}

int jz_destroy(jz_solver* s) {
  if (!s) return JZ_OK;
  (void)hipStreamSynchronize(s->stream);
  destroy_events(s->ev);
  destroy_events(s->ev_free);
  if (s->owns_ws) (void)hipFree(s->ws);
  delete s;
  return JZ_OK;
}

const char* jz_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ===========================================================================
// steps without allocation: the library's static device scratch
// ===========================================================================
// Node-major copies of the state and metrics, stage buffers, partial sums,
// clock and flag of jz_advance_static.  Each GPU the library runs on holds
// its own copy from the time the library's code is loaded there until the
// process ends.  Host code never passes the array's name to a kernel: it
// passes the device address hipGetSymbolAddress gave for the current device.
static __device__ __align__(256) unsigned char scratch[JZ_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on device dev (which is current),
// looked up once per device.
int static_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(JZ_EINVAL, "jz_advance_static: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(JZ_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return JZ_OK;
}

}  // namespace

extern "C" {

int jz_advance_static(int ni, int nj, int nk, const jz_params* p, const double* met, double* q, double* info,
                      int nsteps, void* hip_stream) {
  if (!met || !q) return fail(JZ_EINVAL, "jz_advance_static: NULL argument");
  if (ni < 1 || nj < 1 || nk < 1)
    return fail(JZ_EINVAL, "jz_advance_static: sizes must be >= 1 (got %d %d %d)", ni, nj, nk);
  if (nsteps < 0) return fail(JZ_EINVAL, "jz_advance_static: nsteps < 0");
  if ((long long)ni * nj > (1LL << 30) || (long long)ni * nj * nk > (1LL << 36))
    return fail(JZ_EINVAL, "jz_advance_static: block too large");
  std::string why;
  if (!params_ok(p, &why) || !dims_ok(ni, nj, nk, p, &why))
    return fail(JZ_EINVAL, "jz_advance_static: %s", why.c_str());
  if (p->stats_interval > 0)
    return fail(JZ_EINVAL, "jz_advance_static: time-averaged statistics need a solver (stats_interval must be 0)");
  jz_solver s{};
  setup_shape(&s, ni, nj, nk, p);
  if (s.L.total > JZ_STATIC_SCRATCH_BYTES)
    return fail(JZ_EINVAL, "jz_advance_static: a %dx%dx%d block needs %zu bytes of scratch, the static array holds %zu",
                ni, nj, nk, s.L.total, (size_t)JZ_STATIC_SCRATCH_BYTES);
  HIP_TRY(hipGetDevice(&s.device));
  char* base = nullptr;
  int rc = static_scratch(s.device, &base);
  if (rc) return rc;
  s.ws = base;
  s.owns_ws = false;
  s.stream = (hipStream_t)hip_stream;
  bind_workspace(&s);
  // a run that starts afresh: clock and flag cleared, state and metrics
  // copied into the scratch layout
  HIP_TRY(launch_reset_clock(s.clock, s.flag, s.stream));
  if (s.prec == JZ_FP64)
    HIP_TRY(launch_soa_to_nodes(met, (double*)s.met, s.N, 10, s.stream));
  else
    HIP_TRY(launch_soa_to_met32(met, (float*)s.met, s.jac, s.N, s.stream));
  HIP_TRY(launch_soa_to_nodes(q, s.q0, s.N, 5, s.stream));
  s.grid_set = s.state_set = true;
  rc = advance_steps(&s, nsteps);
  if (rc) return rc;
  HIP_TRY(launch_nodes_to_soa(s.q0, q, s.N, 5, s.stream));
  if (info) HIP_TRY(launch_export_clock(s.clock, s.flag, info, s.stream));
  return JZ_OK;
}

}  // extern "C"

// ===========================================================================
// batches of blocks
// ===========================================================================
struct jz_batch {
  std::vector<jz_solver*> m;
  int prec, ns, bx, by;
  double alpha[5];
  hipStream_t user;
  hipStream_t st;          // internal non-blocking stream (graph capture needs one)
  hipEvent_t ev_in, ev_out;
  BlockDesc* d_desc;       // member table (cap slots)
  int* d_off;              // first global tile of each member (cap + 1)
  BatchCtl* d_ctl;         // work list read by the stage launches
  int cap;                 // member slots of the device tables
  int total;               // tiles of all members
  long long npoints;
  bool use_graph, graph_ok;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;       // recorded, not yet read
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;  // pool filled by jz_batch_set_timing
  double ms_acc;
  long long steps_acc;
  // Pinned staging buffers of the table uploads, each with the event of its
  // last copy: a change of the member set is queued on the batch's stream
  // behind the steps in flight instead of waiting for them.  A buffer is
  // reused only after kStage later changes, so the host waits only when that
  // many changes are queued behind unfinished steps (a server changes the set
  // a few times per chunk of steps; with four buffers the removals of runs
  // finishing together waited for the chunk just queued).
  static constexpr int kStage = 32;
  char* h_stage[kStage];
  hipEvent_t ev_stage[kStage];
  size_t stage_bytes;
  int stage_next;
  hipEvent_t ev_member;    // orders a joining or leaving member's stream against the batch's
};

namespace {

void batch_drop_graph(jz_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_ok = false;
}

// Device tables of the current member set: descriptors, tile offsets and the
// work list (members, tiles, the cost-weighted split among the XCD slots,
// zeroed tile counters).  The captured step reads them from memory, so a
// change of the member set needs no new capture.
// byte offsets of the parts of a staging buffer: work list, tile offsets, descriptors
size_t stage_off_ofs() { return align_up(sizeof(BatchCtl)); }
size_t stage_desc_ofs(int cap) { return align_up(stage_off_ofs() + (cap + 1) * sizeof(int)); }
size_t stage_size(int cap) { return stage_desc_ofs(cap) + cap * sizeof(BlockDesc); }

// The descriptor of a block as the persistent stage launches read it.
void fill_desc(jz_solver* s, BlockDesc& D) {
  D.q0 = s->q0;
  D.bufA = s->prec == JZ_FP64 ? (void*)s->qa : (void*)s->q32a;
  D.bufB = s->prec == JZ_FP64 ? (void*)s->qb : (void*)s->q32b;
  D.met = s->met;
  D.jac = s->jac;
  D.clock = s->clock;
  D.norm_part = s->norm_part;
  D.lam_part = s->lam_part;
  D.flag = s->flag;
  D.N = s->N;
  D.ni = s->ni;
  D.nj = s->nj;
  D.nk = s->nk;
  D.tiles_i = s->tl.tiles_i;
  D.tiles_j = s->tl.tiles_j;
  D.kchunk = s->tl.kchunk;
  D.nchunks = s->tl.nchunks;
  D.ntiles = s->tl.nblocks;
  D.in = s->in;
  D.ctl = step_ctl(s);
  D.ph = s->ph;
}

// The work list of blocks m (tiles member by member, each in its logical
// order) with zeroed counters.  The tile list is split among the slots by
// plane steps: a tile of a chunk of L planes marches L + 2 of them, plus
// about two planes' worth of set-up and reductions.
void fill_worklist(const std::vector<jz_solver*>& m, BatchCtl& c) {
  std::memset(&c, 0, sizeof c);
  c.nblk = (int)m.size();
  auto tile_cost = [](const jz_solver* s, int chunk) {
    const int ek = s->in.hi[2] - s->in.lo[2];
    const int len = std::min(s->tl.kchunk, ek - chunk * s->tl.kchunk);
    return (long long)len + 4;
  };
  long long all = 0;
  for (jz_solver* s : m)
    for (int ch = 0; ch < s->tl.nchunks; ++ch) all += tile_cost(s, ch) * s->tl.tiles_i * s->tl.tiles_j;
  int x = 1, g = 0;
  long long acc = 0;
  for (jz_solver* s : m)
    for (int ch = 0; ch < s->tl.nchunks; ++ch) {
      const long long w = tile_cost(s, ch);
      for (int t = 0; t < s->tl.tiles_i * s->tl.tiles_j; ++t, ++g) {
        while (x < kBatchSlots && acc * kBatchSlots >= all * x) c.split[x++] = g;
        acc += w;
      }
    }
  while (x <= kBatchSlots) c.split[x++] = g;
  c.total = g;
}

int batch_tables(jz_batch* b) {
  const int n = (int)b->m.size();
  const int si = b->stage_next;
  b->stage_next = (si + 1) % jz_batch::kStage;
  HIP_TRY(hipEventSynchronize(b->ev_stage[si]));  // the buffer's previous copy is done
  char* h = b->h_stage[si];
  if (!h) return fail(JZ_ENOMEM, "batch tables: no staging buffer (an earlier allocation failed)");
  BlockDesc* d = reinterpret_cast<BlockDesc*>(h + stage_desc_ofs(b->cap));
  int* off = reinterpret_cast<int*>(h + stage_off_ofs());
  BatchCtl& c = *reinterpret_cast<BatchCtl*>(h);
  off[0] = 0;
  b->npoints = 0;
  for (int i = 0; i < n; ++i) {
    fill_desc(b->m[i], d[i]);
    off[i + 1] = off[i] + b->m[i]->tl.nblocks;
    b->npoints += b->m[i]->N;
  }
  b->total = off[n];
  fill_worklist(b->m, c);
  if (n > 0) HIP_TRY(hipMemcpyAsync(b->d_desc, d, n * sizeof(BlockDesc), hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipMemcpyAsync(b->d_off, off, (n + 1) * sizeof(int), hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipMemcpyAsync(b->d_ctl, &c, sizeof c, hipMemcpyHostToDevice, b->st));
  HIP_TRY(hipEventRecord(b->ev_stage[si], b->st));
  return JZ_OK;
}

// new tables and a new capture (launch shapes changed)
int batch_upload(jz_batch* b) {
  int rc = batch_tables(b);
  batch_drop_graph(b);
  return rc;
}

// Member slots of the device tables: grow to hold `need` members (a new
// capture follows, since the finalize launch covers every slot).
int batch_reserve(jz_batch* b, int need) {
  if (need <= b->cap && b->d_desc) return JZ_OK;
  int cap = b->cap > 0 ? b->cap : 16;
  while (cap < need) cap *= 2;
  if (b->st) HIP_TRY(hipStreamSynchronize(b->st));
  BlockDesc* d = nullptr;
  int* o = nullptr;
  hipError_t e = hipMalloc((void**)&d, cap * sizeof(BlockDesc));
  if (e == hipSuccess) e = hipMalloc((void**)&o, (cap + 1) * sizeof(int));
  if (e != hipSuccess) {
    if (d) (void)hipFree(d);
    return fail(JZ_ENOMEM, "batch tables: %s", hipGetErrorString(e));
  }
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_off) (void)hipFree(b->d_off);
  b->d_desc = d;
  b->d_off = o;
  b->cap = cap;
  batch_drop_graph(b);
  // staging buffers for the new size (the stream sync above finished their copies)
  for (int i = 0; i < jz_batch::kStage; ++i) {
    if (b->h_stage[i]) (void)hipHostFree(b->h_stage[i]);
    b->h_stage[i] = nullptr;
    e = hipHostMalloc((void**)&b->h_stage[i], stage_size(cap), hipHostMallocDefault);
    if (e != hipSuccess) return fail(JZ_ENOMEM, "batch staging: %s", hipGetErrorString(e));
  }
  b->stage_bytes = stage_size(cap);
  return JZ_OK;
}

// What every member of a batch shares.
struct BatchKind {
  int prec, ns, bx, by;
  double alpha[5];
};

BatchKind kind_of(const jz_solver* s) {
  BatchKind k;
  k.prec = s->prec;
  k.ns = s->p.n_stages;
  k.bx = s->tl.bx;
  k.by = s->tl.by;
  for (int i = 0; i < 5; ++i) k.alpha[i] = s->p.rk_alpha[i];
  return k;
}

// A member must match the batch: precision, stages and coefficients, tile
// shape; periodic, without statistics, with grid and state set.
int batch_member_ok(const BatchKind& f, const jz_solver* s, const char* where, int i) {
  if (!s) return fail(JZ_EINVAL, "%s: NULL member %d", where, i);
  if (!s->grid_set || !s->state_set) return fail(JZ_ESTATE, "%s: member %d has no grid or state", where, i);
  if (s->p.n_stages < 2)
    return fail(JZ_EINVAL, "%s: member %d has a single stage (batches need n_stages >= 2)", where, i);
  if (s->prec != f.prec || s->p.n_stages != f.ns || s->tl.bx != f.bx || s->tl.by != f.by)
    return fail(JZ_EINVAL, "%s: member %d differs in precision, stage count or tile shape", where, i);
  for (int k = 0; k < f.ns; ++k)
    if (s->p.rk_alpha[k] != f.alpha[k]) return fail(JZ_EINVAL, "%s: member %d has other stage coefficients", where, i);
  if (s->in.bnd)
    return fail(JZ_EINVAL, "%s: member %d has physical boundaries (batches take periodic blocks)", where, i);
  if (s->stats) return fail(JZ_EINVAL, "%s: member %d collects statistics (not sampled in batches)", where, i);
  return JZ_OK;
}

// one full step of every member on b->st
int batch_step_launches(jz_batch* b) {
  for (int k = 0; k < b->ns; ++k) {
    if (b->prec == JZ_FP64)
      HIP_TRY(launch_stage_batch_fp64(b->d_desc, b->d_off, b->d_ctl, k, b->ns, b->alpha[k], b->bx, b->by, b->st));
    else
      HIP_TRY(launch_stage_batch_fp32(b->d_desc, b->d_off, b->d_ctl, k, b->ns, b->alpha[k], b->bx, b->by, b->st));
  }
  HIP_TRY(launch_finalize_batch(b->d_desc, b->d_ctl, b->cap, b->st));
  return JZ_OK;
}

int batch_ensure_dt(jz_batch* b) {
  for (jz_solver* s : b->m) {
    if (s->dt_valid) continue;
    hipStream_t keep = s->stream;
    s->stream = b->st;
    int rc = ensure_dt(s);
    s->stream = keep;
    if (rc) return rc;
  }
  return JZ_OK;
}

}  // namespace

extern "C" {

int jz_batch_create(jz_solver* const* members, int nmembers, void* hip_stream, jz_batch** out) {
  if (!out) return fail(JZ_EINVAL, "jz_batch_create: out is NULL");
  *out = nullptr;
  if (!members || nmembers < 1) return fail(JZ_EINVAL, "jz_batch_create: no members");
  jz_solver* f = members[0];
  if (!f) return fail(JZ_EINVAL, "jz_batch_create: NULL member");
  const BatchKind kind = kind_of(f);
  for (int i = 0; i < nmembers; ++i) {
    int rc = batch_member_ok(kind, members[i], "jz_batch_create", i);
    if (rc) return rc;
    for (int j = 0; j < i; ++j)
      if (members[j] == members[i]) return fail(JZ_EINVAL, "jz_batch_create: member %d repeated", i);
  }
  const bool shape_ok = f->prec == JZ_FP64 ? batch64_shape_supported(f->tl.bx, f->tl.by)
                                            : batch32_shape_supported(f->tl.bx, f->tl.by);
  if (!shape_ok) return fail(JZ_EINVAL, "jz_batch_create: tile shape %dx%d has no batch kernel", f->tl.ti, f->tl.tj);
  jz_batch* b = new jz_batch();
  b->m.assign(members, members + nmembers);
  b->prec = f->prec;
  b->ns = f->p.n_stages;
  b->bx = f->tl.bx;
  b->by = f->tl.by;
  for (int k = 0; k < 5; ++k) b->alpha[k] = f->p.rk_alpha[k];
  b->user = (hipStream_t)hip_stream;
  b->d_desc = nullptr;
  b->d_off = nullptr;
  b->d_ctl = nullptr;
  b->cap = 0;
  for (int i = 0; i < jz_batch::kStage; ++i) {
    b->h_stage[i] = nullptr;
    b->ev_stage[i] = nullptr;
  }
  b->stage_bytes = 0;
  b->stage_next = 0;
  b->ev_member = nullptr;
  b->use_graph = true;
  b->graph_ok = false;
  b->graph = nullptr;
  b->exec = nullptr;
  b->timing = false;
  b->ms_acc = 0;
  b->steps_acc = 0;
  hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_ctl, sizeof(BatchCtl));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_member, hipEventDisableTiming);
  for (int i = 0; i < jz_batch::kStage; ++i)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_stage[i], hipEventDisableTiming);
  for (jz_solver* s : b->m)
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    jz_batch_destroy(b);
    return fail(JZ_EHIP, "jz_batch_create: %s", hipGetErrorString(e));
  }
  int rc = batch_reserve(b, nmembers);
  if (rc == JZ_OK) rc = batch_upload(b);
  if (rc) {
    jz_batch_destroy(b);
    return rc;
  }
  *out = b;
  return JZ_OK;
}

int jz_batch_add(jz_batch* b, jz_solver* s) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_add: NULL batch");
  if (!s) return fail(JZ_EINVAL, "jz_batch_add: NULL solver");
  for (jz_solver* o : b->m)
    if (o == s) return fail(JZ_EINVAL, "jz_batch_add: already a member");
  BatchKind kind;
  kind.prec = b->prec;
  kind.ns = b->ns;
  kind.bx = b->bx;
  kind.by = b->by;
  for (int k = 0; k < 5; ++k) kind.alpha[k] = b->alpha[k];
  int rc = batch_member_ok(kind, s, "jz_batch_add", (int)b->m.size());
  if (rc) return rc;
  rc = batch_reserve(b, (int)b->m.size() + 1);
  if (rc) return rc;
  // the batch's next steps follow the member's own set-up
  HIP_TRY(hipEventRecord(b->ev_member, s->stream));
  HIP_TRY(hipStreamWaitEvent(b->st, b->ev_member, 0));
  b->m.push_back(s);
  rc = batch_tables(b);
  if (rc) b->m.pop_back();
  return rc;
}

int jz_batch_remove(jz_batch* b, jz_solver* s) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_remove: NULL batch");
  auto it = std::find(b->m.begin(), b->m.end(), s);
  if (it == b->m.end()) return fail(JZ_EINVAL, "jz_batch_remove: not a member");
  // whatever the caller issues next on the member's stream follows the steps
  // queued so far, the last ones that include it
  HIP_TRY(hipEventRecord(b->ev_member, b->st));
  HIP_TRY(hipStreamWaitEvent(s->stream, b->ev_member, 0));
  b->m.erase(it);
  return batch_tables(b);
}

int jz_batch_members(jz_batch* b) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_members: NULL batch");
  return (int)b->m.size();
}

int jz_batch_set_graph(jz_batch* b, int enable) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_set_graph: NULL batch");
  b->use_graph = enable != 0;
  return JZ_OK;
}

int jz_batch_refresh(jz_batch* b) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_refresh: NULL batch");
  // the members' (common) tile shape, checked before anything changes
  int bx = b->bx, by = b->by;
  if (!b->m.empty()) {
    bx = b->m[0]->tl.bx;
    by = b->m[0]->tl.by;
  }
  for (jz_solver* s : b->m)
    if (s->tl.bx != bx || s->tl.by != by) return fail(JZ_EINVAL, "jz_batch_refresh: members differ in tile shape");
  const bool ok = b->prec == JZ_FP64 ? batch64_shape_supported(bx, by) : batch32_shape_supported(bx, by);
  if (!ok) return fail(JZ_EINVAL, "jz_batch_refresh: tile shape has no batch kernel");
  b->bx = bx;
  b->by = by;
  return batch_upload(b);
}

int jz_batch_advance(jz_batch* b, int nsteps) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_advance: NULL batch");
  if (nsteps < 0) return fail(JZ_EINVAL, "jz_batch_advance: nsteps < 0");
  HIP_TRY(hipEventRecord(b->ev_in, b->user));
  HIP_TRY(hipStreamWaitEvent(b->st, b->ev_in, 0));
  int rc = batch_ensure_dt(b);
  if (rc) return rc;
  if (b->use_graph && !b->graph_ok && nsteps > 0) {
    HIP_TRY(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
    rc = batch_step_launches(b);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(JZ_EHIP, "jz_batch_advance: capture: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_ok = true;
  }
  for (int step = 0; step < nsteps; ++step) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->timing) {
      if (b->ev_free.empty()) {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
      } else {
        e0 = b->ev_free.back().first;
        e1 = b->ev_free.back().second;
        b->ev_free.pop_back();
      }
      HIP_TRY(hipEventRecord(e0, b->st));
    }
    if (b->use_graph) {
      HIP_TRY(hipGraphLaunch(b->exec, b->st));
    } else {
      rc = batch_step_launches(b);
      if (rc) return rc;
    }
    if (b->timing) {
      HIP_TRY(hipEventRecord(e1, b->st));
      b->ev.emplace_back(e0, e1);
    }
  }
  for (jz_solver* s : b->m) s->dt_valid = true;
  HIP_TRY(hipEventRecord(b->ev_out, b->st));
  HIP_TRY(hipStreamWaitEvent(b->user, b->ev_out, 0));
  for (jz_solver* s : b->m)
    if (s->stream != b->user) HIP_TRY(hipStreamWaitEvent(s->stream, b->ev_out, 0));
  return JZ_OK;
}

int jz_batch_set_timing(jz_batch* b, int enable) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_set_timing: NULL batch");
  HIP_TRY(hipStreamSynchronize(b->st));
  for (auto& pr : b->ev) b->ev_free.push_back(pr);
  b->ev.clear();
  b->ms_acc = 0;
  b->steps_acc = 0;
  b->timing = enable != 0;
  // event pairs for the steps to come, so that none is created while steps are issued
  while (b->timing && b->ev_free.size() < 256) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(JZ_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    b->ev_free.emplace_back(e0, e1);
  }
  return JZ_OK;
}

int jz_batch_get_timing(jz_batch* b, double* step_ms, long long* steps, long long* points) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_get_timing: NULL batch");
  HIP_TRY(hipStreamSynchronize(b->st));
  for (auto& pr : b->ev) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    b->ms_acc += ms;
    b->steps_acc += 1;
    b->ev_free.push_back(pr);
  }
  b->ev.clear();
  if (step_ms) *step_ms = b->ms_acc;
  if (steps) *steps = b->steps_acc;
  if (points) *points = b->npoints;
  return JZ_OK;
}

int jz_batch_synchronize(jz_batch* b) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_synchronize: NULL batch");
  HIP_TRY(hipStreamSynchronize(b->st));
  return JZ_OK;
}

// Try each candidate launch shape (tile shape with a batch kernel in this
// precision x planes per chunk) for trial_steps steps after one warm-up step,
// keep the fastest, and put every member back to the state and clock it had
// before.  The member states are saved in temporary device buffers.  A cache
// file (one "key tile_i tile_j kchunk ms" line per batch signature) skips the
// trials for a batch seen before.
int jz_batch_autotune(jz_batch* b, int trial_steps, const char* cache_path, int* tile_i, int* tile_j, int* kchunk,
                      double* best_ms) {
  if (!b) return fail(JZ_EINVAL, "jz_batch_autotune: NULL batch");
  if (trial_steps < 1) return fail(JZ_EINVAL, "jz_batch_autotune: trial_steps < 1");
  if (b->m.empty()) return fail(JZ_ESTATE, "jz_batch_autotune: the batch has no members");
  // batch signature: precision, stage count and the sorted member shapes
  std::vector<long long> shapes;
  for (jz_solver* s : b->m) shapes.push_back(((long long)s->ni << 40) | ((long long)s->nj << 20) | s->nk);
  std::sort(shapes.begin(), shapes.end());
  unsigned long long h = 1469598103934665603ull;
  for (long long v : shapes) h = (h ^ (unsigned long long)v) * 1099511628211ull;
  char key[64];
  snprintf(key, sizeof key, "p%d-s%d-n%zu-%016llx", b->prec, b->ns, b->m.size(), h);
  int best_ti = -1, best_tj = -1, best_kc = -1;
  double best = 1e300;
  if (cache_path) {
    FILE* fp = fopen(cache_path, "r");
    if (fp) {
      char k[64];
      int a1, a2, a3;
      double ms;
      while (fscanf(fp, "%63s %d %d %d %lf", k, &a1, &a2, &a3, &ms) == 5)
        if (strcmp(k, key) == 0) {
          best_ti = a1;
          best_tj = a2;
          best_kc = a3;
          best = ms;
        }
      fclose(fp);
    }
  }
  if (best_ti < 0) {
    std::vector<std::pair<int, int>> cand;
    if (b->prec == JZ_FP64)
      cand = {{16, 12}, {32, 8}, {16, 16}, {28, 12}, {12, 12}};
    else
      cand = {{32, 16}, {28, 20}, {28, 12}, {12, 12}};
    const int kcs[3] = {16, 32, 64};
    // save states and clocks
    std::vector<double*> qsave(b->m.size(), nullptr);
    std::vector<Clock> csave(b->m.size());
    HIP_TRY(hipStreamSynchronize(b->st));
    int rc = JZ_OK;
    for (size_t i = 0; i < b->m.size() && rc == JZ_OK; ++i) {
      jz_solver* s = b->m[i];
      if (hipMalloc((void**)&qsave[i], 5 * s->N * sizeof(double)) != hipSuccess) rc = fail(JZ_ENOMEM, "autotune save");
      if (rc == JZ_OK && hipMemcpy(qsave[i], s->q0, 5 * s->N * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess)
        rc = fail(JZ_EHIP, "autotune save copy");
      if (rc == JZ_OK && hipMemcpy(&csave[i], s->clock, sizeof(Clock), hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(JZ_EHIP, "autotune clock copy");
    }
    auto restore = [&]() -> int {
      for (size_t i = 0; i < b->m.size(); ++i) {
        jz_solver* s = b->m[i];
        if (!qsave[i]) continue;
        HIP_TRY(hipMemcpy(s->q0, qsave[i], 5 * s->N * sizeof(double), hipMemcpyDeviceToDevice));
        HIP_TRY(hipMemcpy(s->clock, &csave[i], sizeof(Clock), hipMemcpyHostToDevice));
        const int z = 0;
        HIP_TRY(hipMemcpy(s->flag, &z, sizeof z, hipMemcpyHostToDevice));
        s->dt_valid = false;
      }
      return JZ_OK;
    };
    const bool timing_was = b->timing;
    for (size_t c = 0; c < cand.size() && rc == JZ_OK; ++c)
      for (int kk = 0; kk < 3 && rc == JZ_OK; ++kk) {
        bool ok = true;
        for (jz_solver* s : b->m)
          if (jz_set_tiling(s, cand[c].first, cand[c].second, kcs[kk]) != JZ_OK) ok = false;
        if (!ok) continue;
        rc = batch_upload(b);
        b->bx = cand[c].first + 4;
        b->by = cand[c].second + 4;
        if (rc == JZ_OK) rc = jz_batch_set_timing(b, 0);
        if (rc == JZ_OK) rc = jz_batch_advance(b, 1);
        if (rc == JZ_OK) rc = jz_batch_set_timing(b, 1);
        if (rc == JZ_OK) rc = jz_batch_advance(b, trial_steps);
        double ms = 0;
        long long n = 0;
        if (rc == JZ_OK) rc = jz_batch_get_timing(b, &ms, &n, nullptr);
        if (rc == JZ_OK && n > 0 && ms / n < best) {
          best = ms / n;
          best_ti = cand[c].first;
          best_tj = cand[c].second;
          best_kc = kcs[kk];
        }
        if (rc == JZ_OK) rc = restore();
      }
    if (rc) (void)restore();  // a failed trial leaves the states as they were
    jz_batch_set_timing(b, timing_was ? 1 : 0);
    for (double* p : qsave)
      if (p) (void)hipFree(p);
    if (rc) return rc;
    if (best_ti < 0) return fail(JZ_EINVAL, "jz_batch_autotune: no candidate shape fits the members");
    if (cache_path) {
      FILE* fp = fopen(cache_path, "a");
      if (fp) {
        fprintf(fp, "%s %d %d %d %.6f\n", key, best_ti, best_tj, best_kc, best);
        fclose(fp);
      }
    }
  }
  // apply the choice to every member, or to none (a cached choice that a
  // member does not take leaves the batch as it was)
  std::vector<std::pair<jz_params, Tiling>> old;
  for (jz_solver* s : b->m) old.emplace_back(s->p, s->tl);
  for (size_t i = 0; i < b->m.size(); ++i) {
    int rc = jz_set_tiling(b->m[i], best_ti, best_tj, best_kc);
    if (rc) {
      for (size_t j = 0; j < i; ++j) {
        b->m[j]->p = old[j].first;
        b->m[j]->tl = old[j].second;
      }
      return rc;
    }
  }
  b->bx = best_ti + 4;
  b->by = best_tj + 4;
  int rc = batch_upload(b);
  if (rc) return rc;
  if (tile_i) *tile_i = best_ti;
  if (tile_j) *tile_j = best_tj;
  if (kchunk) *kchunk = best_kc;
  if (best_ms) *best_ms = best;
  return JZ_OK;
}

int jz_batch_destroy(jz_batch* b) {
  if (!b) return JZ_OK;
  if (b->st) (void)hipStreamSynchronize(b->st);
  for (auto& pr : b->ev) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  batch_drop_graph(b);
  for (auto& pr : b->ev_free) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_off) (void)hipFree(b->d_off);
  if (b->d_ctl) (void)hipFree(b->d_ctl);
  for (int i = 0; i < jz_batch::kStage; ++i) {
    if (b->h_stage[i]) (void)hipHostFree(b->h_stage[i]);
    if (b->ev_stage[i]) (void)hipEventDestroy(b->ev_stage[i]);
  }
  if (b->ev_member) (void)hipEventDestroy(b->ev_member);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->st) (void)hipStreamDestroy(b->st);
  delete b;
  return JZ_OK;
}

}  // extern "C"

// ===========================================================================
// domains: one periodic block split into sub-blocks along xi and zeta, each
// padded with two ghost layers along its split directions that halo copies
// refill after every stage (the paper's decomposition, Sec. 4.1, and its
// two-layer ghost exchange, Sec. 4.3, on one device)
// ===========================================================================
struct jz_domain {
  int n[3];
  int parts[3];                  // sub-blocks per direction (parts[1] = 1)
  std::vector<int> off[3], len[3];  // per direction: first node and node count of each part
  std::vector<jz_solver*> sub;   // part (a, c) (xi index a, zeta index c) at a + parts[0] * c
  jz_params p;
  hipStream_t stream;
  DomainSub* d_sub;              // device table for the group reductions
  int halo;                      // bit d: direction d is split
  long long n_interior;
  bool dt_valid;
  // One persistent launch per stage over the tiles of all parts (FP64, when
  // the parts' tile shape has a batch kernel), and one launch per exchange pass:
  // the parts' descriptors, tile offsets and work list, and the ghost
  // refills of each pass (xi, zeta) for the stage outputs of each kind
  // (0: buffer A, 1: buffer B, 2: Q(0)), stored one after another.
  bool batched;
  int bx, by;
  BlockDesc* d_desc;
  int* d_off;
  BatchCtl* d_ctl;
  HaloJob* d_jobs;
  int job_off[3][2], njobs[3][2];
  long long job_max[3][2];  // threads of the largest job of each pass
  double* d_red;            // [parts][11]: per-part norm sums, maxima, spectral radius
};

namespace {

int dom_index(const jz_domain* D, int a, int c) { return a + D->parts[0] * c; }

// padded extent of part a along d
int dom_pad(const jz_domain* D, int d, int a) { return D->len[d][a] + ((D->halo >> d) & 1 ? 4 : 0); }

// Copy the padded region of part (a, c) out of a whole-block SoA host array
// of `rows` rows (periodic wrap), or back into it (interior nodes only).
void dom_extract(const jz_domain* D, int a, int c, const double* whole, int rows, std::vector<double>& out) {
  const int sn[3] = {dom_pad(D, 0, a), D->n[1], dom_pad(D, 2, c)};
  const int o[3] = {D->off[0][a] - ((D->halo & 1) ? 2 : 0), 0, D->off[2][c] - ((D->halo & 4) ? 2 : 0)};
  const long long N = (long long)D->n[0] * D->n[1] * D->n[2], sN = (long long)sn[0] * sn[1] * sn[2];
  out.assign((size_t)rows * sN, 0.0);
  for (int k = 0; k < sn[2]; ++k)
    for (int j = 0; j < sn[1]; ++j)
      for (int i = 0; i < sn[0]; ++i) {
        const long long g = wrap_index(o[0] + i, D->n[0]) +
                            (long long)D->n[0] * (j + (long long)D->n[1] * wrap_index(o[2] + k, D->n[2]));
        const long long l = i + (long long)sn[0] * (j + (long long)sn[1] * k);
        for (int r = 0; r < rows; ++r) out[r * sN + l] = whole[r * N + g];
      }
}

void dom_insert(const jz_domain* D, int a, int c, const std::vector<double>& part, double* whole) {
  const int sn[3] = {dom_pad(D, 0, a), D->n[1], dom_pad(D, 2, c)};
  const int g0[3] = {(D->halo & 1) ? 2 : 0, 0, (D->halo & 4) ? 2 : 0};
  const long long N = (long long)D->n[0] * D->n[1] * D->n[2], sN = (long long)sn[0] * sn[1] * sn[2];
  for (int k = 0; k < D->len[2][c]; ++k)
    for (int j = 0; j < D->n[1]; ++j)
      for (int i = 0; i < D->len[0][a]; ++i) {
        const long long g = (D->off[0][a] + i) + (long long)D->n[0] * (j + (long long)D->n[1] * (D->off[2][c] + k));
        const long long l = (g0[0] + i) + (long long)sn[0] * (j + (long long)sn[1] * (g0[2] + k));
        for (int r = 0; r < 5; ++r) whole[r * N + g] = part[r * sN + l];
      }
}

// The stage output buffer of stage k (as jz_advance rotates them).
void* dom_stage_out(jz_solver* s, int k, int ns) {
  if (k == ns - 1) return s->q0;
  const bool f32 = s->prec == JZ_FP32_FLUX;
  return (k % 2 == 0) ? (f32 ? (void*)s->q32a : (void*)s->qa) : (f32 ? (void*)s->q32b : (void*)s->qb);
}

// kind of the stage output of stage k: 0 buffer A, 1 buffer B, 2 Q(0)
int dom_kind(int k, int ns) { return k == ns - 1 ? 2 : (k % 2); }

// Refill the ghost layers of every part's buffer of stage k: first along xi
// (all zeta planes), then along zeta over the whole padded width, which
// carries the xi ghost columns -- and with them the corners -- across.  One
// launch per split direction over that pass's table of copy jobs.
int dom_exchange(jz_domain* D, int k, int ns) {
  const bool f32 = D->p.precision == JZ_FP32_FLUX && k != ns - 1;
  const int kind = dom_kind(k, ns);
  for (int pass = 0; pass < 2; ++pass) {
    const int d = pass == 0 ? 0 : 2;
    if (!((D->halo >> d) & 1)) continue;
    HIP_TRY(launch_halo_jobs(D->d_jobs + D->job_off[kind][pass], D->njobs[kind][pass], f32, d,
                             D->job_max[kind][pass], D->stream));
  }
  return JZ_OK;
}

// The ghost refills of every pass and stage-output kind, and, when the
// parts' tile shape has a batch kernel, their batch tables.
int dom_build_launch_tables(jz_domain* D) {
  std::vector<HaloJob> jobs;
  for (int kind = 0; kind < 3; ++kind)
    for (int pass = 0; pass < 2; ++pass) {
      const int d = pass == 0 ? 0 : 2;
      D->job_off[kind][pass] = (int)jobs.size();
      D->njobs[kind][pass] = 0;
      D->job_max[kind][pass] = 0;
      if (!((D->halo >> d) & 1)) continue;
      for (int c = 0; c < D->parts[2]; ++c)
        for (int a = 0; a < D->parts[0]; ++a) {
          jz_solver* dst = D->sub[dom_index(D, a, c)];
          const int np = D->parts[d], pos = d == 0 ? a : c;
          const int prev = (pos + np - 1) % np, next = (pos + 1) % np;
          jz_solver* lo = D->sub[d == 0 ? dom_index(D, prev, c) : dom_index(D, a, prev)];
          jz_solver* hi = D->sub[d == 0 ? dom_index(D, next, c) : dom_index(D, a, next)];
          auto buf = [&](jz_solver* s) -> void* {
            const bool f32 = s->prec == JZ_FP32_FLUX;
            if (kind == 2) return s->q0;
            return kind == 0 ? (f32 ? (void*)s->q32a : (void*)s->qa) : (f32 ? (void*)s->q32b : (void*)s->qb);
          };
          for (int side = 0; side < 2; ++side) {
            jz_solver* src = side == 0 ? lo : hi;
            HaloJob J;
            J.dst = buf(dst);
            J.src = buf(src);
            J.nd[0] = dst->ni;
            J.nd[1] = dst->nj;
            J.nd[2] = dst->nk;
            J.nsrc[0] = src->ni;
            J.nsrc[1] = src->nj;
            J.nsrc[2] = src->nk;
            // low ghosts <- the last two own layers of the lower part; high
            // ghosts <- the first two own layers of the upper part
            J.dl0 = side == 0 ? 0 : J.nd[d] - 2;
            J.sl0 = side == 0 ? J.nsrc[d] - 4 : 2;
            jobs.push_back(J);
            // ten threads per ghost row along xi, one per value otherwise
            const long long cnt = d == 0 ? 10LL * J.nd[1] * J.nd[2] : 2LL * J.nd[face_e(d)] * J.nd[face_f(d)] * 5;
            if (cnt > D->job_max[kind][pass]) D->job_max[kind][pass] = cnt;
            D->njobs[kind][pass] += 1;
          }
        }
    }
  if (!jobs.empty()) {
    HIP_TRY(hipMalloc((void**)&D->d_jobs, jobs.size() * sizeof(HaloJob)));
    HIP_TRY(hipMemcpy(D->d_jobs, jobs.data(), jobs.size() * sizeof(HaloJob), hipMemcpyHostToDevice));
  }
  // Batched stage launches (FP64): every part shares the tile shape.  The
  // FP32-flux batch kernel keeps the primitive ring and reads the metrics
  // again in its first and last stages, which costs more than the tails of
  // one launch per part (split 2 x 2 at 512 x 256 x 256: 11 % against 10 %
  // over the unsplit block); in FP64 the batched launch took the overhead
  // from 13 % to 6 % (5 % with the row-wise xi copies and the two-level
  // step reductions).
  D->bx = D->sub[0]->tl.bx;
  D->by = D->sub[0]->tl.by;
  bool same = true;
  for (jz_solver* s : D->sub) same = same && s->tl.bx == D->bx && s->tl.by == D->by;
  D->batched = same && D->p.precision == JZ_FP64 && batch64_shape_supported(D->bx, D->by);
  if (!D->batched) return JZ_OK;
  const int n = (int)D->sub.size();
  std::vector<BlockDesc> desc(n);
  std::vector<int> off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    fill_desc(D->sub[i], desc[i]);
    off[i + 1] = off[i] + D->sub[i]->tl.nblocks;
  }
  BatchCtl c;
  fill_worklist(D->sub, c);
  HIP_TRY(hipMalloc((void**)&D->d_desc, n * sizeof(BlockDesc)));
  HIP_TRY(hipMalloc((void**)&D->d_off, (n + 1) * sizeof(int)));
  HIP_TRY(hipMalloc((void**)&D->d_ctl, sizeof(BatchCtl)));
  HIP_TRY(hipMemcpy(D->d_desc, desc.data(), n * sizeof(BlockDesc), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->d_off, off.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(D->d_ctl, &c, sizeof c, hipMemcpyHostToDevice));
  return JZ_OK;
}

int dom_upload_table(jz_domain* D) {
  std::vector<DomainSub> t(D->sub.size());
  for (size_t i = 0; i < D->sub.size(); ++i) {
    jz_solver* s = D->sub[i];
    t[i].clock = s->clock;
    t[i].norm_part = s->norm_part;
    t[i].lam_part = s->lam_part;
    t[i].flag = s->flag;
    t[i].nb_tiles = s->tl.nblocks;
    t[i].nb_lmax = lambda_max_blocks(s->N);
  }
  HIP_TRY(hipMemcpyAsync(D->d_sub, t.data(), t.size() * sizeof(DomainSub), hipMemcpyHostToDevice, D->stream));
  HIP_TRY(hipStreamSynchronize(D->stream));
  return JZ_OK;
}

StepCtl dom_ctl(const jz_domain* D) {
  StepCtl c;
  c.cfl = D->p.cfl;
  c.dt_fixed = D->p.dt_fixed;
  c.inv_n = 1.0 / (double)D->n_interior;
  return c;
}

int dom_ensure_dt(jz_domain* D) {
  if (D->dt_valid) return JZ_OK;
  for (jz_solver* s : D->sub) {
    const int n[3] = {s->ni, s->nj, s->nk};
    HIP_TRY(launch_lambda_max(s->q0, s->met, s->jac, s->prec == JZ_FP32_FLUX, s->N, n, s->in, s->p.gamma,
                              s->lam_part, D->stream));
  }
  HIP_TRY(launch_domain_dt(D->d_sub, (int)D->sub.size(), dom_ctl(D), D->stream));
  // the parts' clocks hold the common dt now (their own getters must not replace it)
  for (jz_solver* s : D->sub) s->dt_valid = true;
  D->dt_valid = true;
  return JZ_OK;
}

}  // namespace

extern "C" {

int jz_domain_create(int ni, int nj, int nk, const jz_params* p, int parts_i, int parts_k, void* hip_stream,
                     jz_domain** out) {
  if (!out) return fail(JZ_EINVAL, "jz_domain_create: out is NULL");
  *out = nullptr;
  std::string why;
  if (!params_ok(p, &why)) return fail(JZ_EINVAL, "jz_domain_create: %s", why.c_str());
  if (bounded_mask(p) || p->stats_interval > 0 || p->n_stages < 2)
    return fail(JZ_EINVAL, "jz_domain_create: domains take periodic blocks without statistics and with n_stages >= 2");
  if (parts_i < 1 || parts_k < 1 || ni < 2 * parts_i || nk < 2 * parts_k || nj < 1)
    return fail(JZ_EINVAL, "jz_domain_create: every part needs at least 2 nodes along a split direction");
  if ((long long)ni * nj * nk > (1LL << 36)) return fail(JZ_EINVAL, "jz_domain_create: block too large");
  jz_domain* D = new jz_domain();
  D->n[0] = ni;
  D->n[1] = nj;
  D->n[2] = nk;
  D->parts[0] = parts_i;
  D->parts[1] = 1;
  D->parts[2] = parts_k;
  D->halo = (parts_i > 1 ? 1 : 0) | (parts_k > 1 ? 4 : 0);
  D->p = *p;
  D->stream = (hipStream_t)hip_stream;
  D->d_sub = nullptr;
  D->n_interior = (long long)ni * nj * nk;
  D->dt_valid = false;
  D->batched = false;
  D->bx = D->by = 0;
  D->d_desc = nullptr;
  D->d_off = nullptr;
  D->d_ctl = nullptr;
  D->d_jobs = nullptr;
  D->d_red = nullptr;
  // balanced parts: sizes differ by at most one node, larger ones first
  for (int d = 0; d < 3; ++d) {
    const int np = D->parts[d];
    int o = 0;
    for (int a = 0; a < np; ++a) {
      const int l = D->n[d] / np + (a < D->n[d] % np ? 1 : 0);
      D->off[d].push_back(o);
      D->len[d].push_back(l);
      o += l;
    }
  }
  for (int c = 0; c < parts_k; ++c)
    for (int a = 0; a < parts_i; ++a) {
      jz_params sp = *p;
      jz_solver* s = nullptr;
      const int sn[3] = {dom_pad(D, 0, a), nj, dom_pad(D, 2, c)};
      int rc = jz_create(sn[0], sn[1], sn[2], &sp, nullptr, 0, hip_stream, &s);
      if (rc) {
        jz_domain_destroy(D);
        return rc;
      }
      // the split directions: advance [2, n - 2), ghost layers read, not wrapped
      Interior in = s->in;
      for (int d = 0; d < 3; ++d)
        if ((D->halo >> d) & 1) {
          in.bnd |= 1 << d;
          in.lo[d] = 2;
          in.hi[d] = sn[d] - 2;
        }
      s->in = in;
      pick_tiling_for_device(sn[0], sn[1], sn[2], &sp, &s->tl, &in);
      D->sub.push_back(s);
    }
  // The FP64 parts of the compact shape run in one batched launch per stage,
  // so their chunks are chosen for the domain as a whole: 64 planes when all
  // the parts' tiles fill the device with them.  A part on its own would take
  // shorter chunks to fill the device and march more warm-up planes (4 x 4
  // parts of 512 x 256 x 256: 13 instead of 64 planes, 13 % longer stages).
  if (p->precision == JZ_FP64 && p->kchunk <= 0) {
    bool compact = true;
    long long tiles = 0;
    for (jz_solver* s : D->sub) {
      const int ek = s->in.hi[2] - s->in.lo[2];
      compact = compact && s->tl.bx == 20 && s->tl.by == 16;
      tiles += (long long)s->tl.tiles_i * s->tl.tiles_j * ((ek + 63) / 64);
    }
    int dev = 0, ncu = 0;
    if (compact && hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        tiles >= (long long)stage_wg_per_cu_fp64(20, 16) * ncu) {
      for (jz_solver* s : D->sub) {
        const int ek = s->in.hi[2] - s->in.lo[2];
        Tiling& t = s->tl;
        t.kchunk = ek < 64 ? ek : 64;
        t.nchunks = (ek + t.kchunk - 1) / t.kchunk;
        t.nblocks = t.tiles_i * t.tiles_j * t.nchunks;
      }
    }
  }
  hipError_t e = hipMalloc((void**)&D->d_sub, D->sub.size() * sizeof(DomainSub));
  if (e == hipSuccess) e = hipMalloc((void**)&D->d_red, D->sub.size() * 11 * sizeof(double));
  if (e != hipSuccess) {
    jz_domain_destroy(D);
    return fail(JZ_ENOMEM, "jz_domain_create: %s", hipGetErrorString(e));
  }
  int rc = dom_upload_table(D);
  if (rc == JZ_OK) rc = dom_build_launch_tables(D);
  if (rc) {
    jz_domain_destroy(D);
    return rc;
  }
  *out = D;
  return JZ_OK;
}

int jz_domain_set_grid_metrics(jz_domain* D, const double* m) {
  if (!D || !m) return fail(JZ_EINVAL, "jz_domain_set_grid_metrics: NULL argument");
  std::vector<double> part;
  for (int c = 0; c < D->parts[2]; ++c)
    for (int a = 0; a < D->parts[0]; ++a) {
      dom_extract(D, a, c, m, 10, part);
      int rc = jz_set_grid_metrics(D->sub[dom_index(D, a, c)], part.data(), 0);
      if (rc) return rc;
    }
  D->dt_valid = false;
  return JZ_OK;
}

int jz_domain_set_state(jz_domain* D, const double* q) {
  if (!D || !q) return fail(JZ_EINVAL, "jz_domain_set_state: NULL argument");
  std::vector<double> part;
  for (int c = 0; c < D->parts[2]; ++c)
    for (int a = 0; a < D->parts[0]; ++a) {
      dom_extract(D, a, c, q, 5, part);
      int rc = jz_set_state(D->sub[dom_index(D, a, c)], part.data(), 0);
      if (rc) return rc;
    }
  D->dt_valid = false;
  return JZ_OK;
}

int jz_domain_advance(jz_domain* D, int nsteps) {
  if (!D) return fail(JZ_EINVAL, "jz_domain_advance: NULL domain");
  if (nsteps < 0) return fail(JZ_EINVAL, "jz_domain_advance: nsteps < 0");
  for (jz_solver* s : D->sub)
    if (!s->grid_set || !s->state_set) return fail(JZ_ESTATE, "jz_domain_advance: grid and state must be set first");
  int rc = dom_ensure_dt(D);
  if (rc) return rc;
  const int ns = D->p.n_stages;
  for (int step = 0; step < nsteps; ++step) {
    for (int k = 0; k < ns; ++k) {
      if (D->batched) {
        // one persistent launch over the tiles of every part
        const double alpha = D->p.rk_alpha[k];
        HIP_TRY(launch_stage_batch_fp64(D->d_desc, D->d_off, D->d_ctl, k, ns, alpha, D->bx, D->by, D->stream));
      } else {
        for (jz_solver* s : D->sub) {
          const void* in = k == 0 ? (const void*)s->q0 : dom_stage_out(s, k - 1, ns);
          StageArgs a = stage_args(s, in, dom_stage_out(s, k, ns), s->p.rk_alpha[k]);
          HIP_TRY(launch_stage(s, a, k, ns, false));
        }
      }
      rc = dom_exchange(D, k, ns);
      if (rc) return rc;
    }
    HIP_TRY(launch_domain_finalize(D->d_sub, (int)D->sub.size(), dom_ctl(D), D->batched ? D->d_ctl : nullptr,
                                   D->d_red, D->stream));
  }
  return JZ_OK;
}

int jz_domain_get_state(jz_domain* D, double* q) {
  if (!D || !q) return fail(JZ_EINVAL, "jz_domain_get_state: NULL argument");
  std::vector<double> part;
  int status = JZ_OK;
  for (int c = 0; c < D->parts[2]; ++c)
    for (int a = 0; a < D->parts[0]; ++a) {
      jz_solver* s = D->sub[dom_index(D, a, c)];
      part.assign(5 * (size_t)s->N, 0.0);
      int rc = jz_get_state(s, part.data(), 0);
      if (rc && rc != JZ_ENONFINITE) return rc;
      if (rc) status = rc;
      dom_insert(D, a, c, part, q);
    }
  return status;
}

int jz_domain_get_clock(jz_domain* D, double* t, double* next_dt, long long* steps) {
  if (!D) return fail(JZ_EINVAL, "jz_domain_get_clock: NULL domain");
  int rc = dom_ensure_dt(D);
  if (rc) return rc;
  return jz_get_clock(D->sub[0], t, next_dt, steps);
}

int jz_domain_get_residual_norms(jz_domain* D, double rms[5], double linf[5]) {
  if (!D) return fail(JZ_EINVAL, "jz_domain_get_residual_norms: NULL domain");
  return jz_get_residual_norms(D->sub[0], rms, linf);
}

int jz_domain_destroy(jz_domain* D) {
  if (!D) return JZ_OK;
  if (D->stream) (void)hipStreamSynchronize(D->stream);
  for (jz_solver* s : D->sub) jz_destroy(s);
  if (D->d_sub) (void)hipFree(D->d_sub);
  if (D->d_desc) (void)hipFree(D->d_desc);
  if (D->d_off) (void)hipFree(D->d_off);
  if (D->d_ctl) (void)hipFree(D->d_ctl);
  if (D->d_jobs) (void)hipFree(D->d_jobs);
  if (D->d_red) (void)hipFree(D->d_red);
  delete D;
  return JZ_OK;
}

}  // extern "C"
