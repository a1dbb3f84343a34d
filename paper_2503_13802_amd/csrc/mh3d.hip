// Host side of the MH3D C ABI (include/mh3d.h): plan construction, launch-shape
// selection with host-side fit checks, operator application, power iteration and
// the accelerated projected gradient solver (paper Sec. 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mh3d.h"
#include "kernels.hpp"
#include "fast.hpp"

using namespace mh3d;

// ============================================================================ errors
static thread_local std::string g_err = "no error";

static mh3d_status fail(mh3d_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define CHK(x)                          \
  do {                                  \
    mh3d_status s_ = (x);               \
    if (s_ != MH3D_OK) return s_;       \
  } while (0)

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(MH3D_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                 \
  } while (0)

extern "C" const char* mh3d_last_error(void) { return g_err.c_str(); }
extern "C" int32_t mh3d_version(void) { return MH3D_VERSION_MAJOR * 100 + MH3D_VERSION_MINOR; }

// ============================================================================ geometry
static bool is_23_smooth(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

static const size_t kLdsLimit = 160 * 1024;

struct Launch {
  int T_plane, T_class, T_small;
  // threads per block of k_adj_and_store (512 or 1024; both bodies loop over blockDim):
  // with 512 two blocks share a CU, so more small-grid blocks run beside the plane blocks
  int T_merge;
  size_t lds_plane, lds_class, lds_small;
};

// A class-kernel element split e is valid when it is one of the compiled splits
// (1, 2, 3, 4, 6, 8, 9), divides S, and S/e is a power of two <= 64 (the fold
// reduction then stays inside aligned lane groups).
static bool valid_E(int S, int e) {
  if (!(e == 1 || e == 2 || e == 3 || e == 4 || e == 6 || e == 8 || e == 9)) return false;
  if (S % e) return false;
  const int lg = S / e;
  return lg <= 64 && (lg & (lg - 1)) == 0;
}

// Tile shapes of the class and small-grid kernels: E elements per thread and cpw
// classes per workgroup (class passes), xb x' planes per workgroup (small-grid
// passes).  A value <= 0 asks for the built-in heuristic.  Fills the derived fields
// of g and L; fails if a requested shape is invalid or does not fit.
static mh3d_status derive_tiles(Geo& g, Launch& L, int E_req, int cpw_req, int xb_req, int ps_req) {
  // ---- class kernel: E so the launch has enough waves in flight, then cpw
  if (E_req > 0) {
    if (!valid_E(g.S, E_req)) return fail(MH3D_ERR_INVALID, "E = %d is not a valid split of S = %d", E_req, g.S);
    g.E = E_req;
  } else {
    g.E = -1;
    const int opts[7] = {8, 6, 4, 3, 2, 1, 9};
    const long elems = (long)g.ncls * g.mx * g.S;
    int fallback = -1;
    for (int e : opts) {
      if (!valid_E(g.S, e)) continue;
      if (fallback < 0 || e < fallback) fallback = e;
      if (elems / e >= 128 * 1024 && g.E < 0) g.E = e;
    }
    if (g.E < 0) g.E = fallback;
    if (g.E < 0) return fail(MH3D_ERR_UNSUPPORTED, "decimation product %d has no supported fold split", g.S);
  }
  if (cpw_req > 0) {
    if (g.ncls % cpw_req) return fail(MH3D_ERR_INVALID, "cpw = %d does not divide %d classes", cpw_req, g.ncls);
    const long T = (long)cpw_req * g.mx * g.S / g.E;
    Geo t = g;
    t.cpw = cpw_req;
    if (T > 1024 || class_lds_elems(t) * sizeof(float2) > 64 * 1024)
      return fail(MH3D_ERR_INVALID, "cpw = %d gives %ld threads / too much LDS", cpw_req, T);
    g.cpw = cpw_req;
  } else {
    int best_cpw = 0;
    for (int c = 1; c <= g.ncls; ++c) {
      if (g.ncls % c) continue;
      const long T = (long)c * g.mx * g.S / g.E;
      if (T > 1024) break;
      Geo t = g;
      t.cpw = c;
      if (class_lds_elems(t) * sizeof(float2) > 64 * 1024) break;
      best_cpw = c;
      if (T >= 128 && T % 64 == 0) break;
    }
    if (!best_cpw) return fail(MH3D_ERR_UNSUPPORTED, "no class-kernel shape fits (mx*S/E or LDS too large)");
    g.cpw = best_cpw;
  }
  L.T_class = g.cpw * g.mx * g.S / g.E;
  L.lds_class = class_lds_elems(g) * sizeof(float2);

  // ---- small kernel: x' planes per workgroup (aim for >= 256 workgroups)
  if (xb_req > 0) {
    if (g.mx % xb_req || xb_req > 64) return fail(MH3D_ERR_INVALID, "xb = %d does not divide mx = %d", xb_req, g.mx);
    g.xb = xb_req;
  } else {
    g.xb = 1;
    for (int xb : {8, 4, 2, 1}) {
      if (g.mx % xb) continue;
      if ((long)g.K * (g.mx / xb) >= 256 || xb == 1) { g.xb = xb; break; }
    }
  }
  g.spairs = (g.xb * g.my + 1) / 2;
  // ---- plane passes: workgroups per x-plane (2 unless asked otherwise; each takes a
  // share of the columns / row pairs, so at most min(nz/2 + 1, (ny + 1)/2) of them)
  if (ps_req > 4 || ps_req > g.nzh || ps_req > g.npairs)
    return fail(MH3D_ERR_INVALID, "ps = %d: the plane passes take 1 to 4 workgroups per plane (at most "
                "min(nz/2+1, (ny+1)/2))", ps_req);
  g.ps = ps_req > 0 ? ps_req : std::min(2, std::min(g.nzh, g.npairs));
  g.f_nz = make_fastdiv(g.nz); g.f_nzh = make_fastdiv(g.nzh); g.f_nmem = make_fastdiv(g.nmem);
  g.f_mzh = make_fastdiv(g.mzh); g.f_sz = make_fastdiv(g.sz); g.f_mz = make_fastdiv(g.mz);
  g.f_W = make_fastdiv(g.cpw * g.nmem); g.f_xb = make_fastdiv(g.xb); g.f_S = make_fastdiv(g.S);
  g.f_mxS = make_fastdiv(g.mx * g.S); g.f_cpwmx = make_fastdiv(g.cpw * g.mx);
  g.f_cpwxb = make_fastdiv(g.cpw * g.xb); g.f_ny = make_fastdiv(g.ny); g.f_my = make_fastdiv(g.my);
  // 256 threads per decimated x'-plane of the block (the small-grid kernels loop over
  // blockDim, so the count only sets how much of the block's work runs side by side)
  L.T_small = std::min(1024, 256 * g.xb);
  L.T_merge = g.ps >= 2 ? 512 : 1024;   // the autotuner times both
  L.lds_small = sizeof(float2) * ((size_t)g.my + g.mz + 2 * (size_t)small_lds(g));
  if (L.lds_small > kLdsLimit) return fail(MH3D_ERR_UNSUPPORTED, "small-grid plane does not fit in LDS");
  return MH3D_OK;
}

static mh3d_status build_geo(const mh3d_plan_desc* d, Geo& g, Launch& L, const mh3d_tiles* tiles = nullptr) {
  if (!d) return fail(MH3D_ERR_INVALID, "descriptor is NULL");
  const int n[3] = {d->nx, d->ny, d->nz};
  // ny = 1: a 2D image [nx][1][nz], the projection axis of the 2D geometry (Sec. 5.2)
  const bool flat = d->ny == 1;
  for (int a = 0; a < 3; ++a) {
    if (a == 1 && flat) {
      if (d->ds[1] != 1) return fail(MH3D_ERR_INVALID, "a 2D grid (ny = 1) needs ds[1] = 1");
      if (d->pad[1] != 0) return fail(MH3D_ERR_INVALID, "a 2D grid (ny = 1) has no padding along y");
      continue;
    }
    if (n[a] < 4 || n[a] > 256 || !is_23_smooth(n[a]))
      return fail(MH3D_ERR_INVALID, "grid axis %d = %d must be 2^a 3^b in [4, 256] (ny may be 1)", a, n[a]);
    if (d->ds[a] < 1 || n[a] % d->ds[a])
      return fail(MH3D_ERR_INVALID, "decimation ds[%d] = %d must divide %d", a, d->ds[a], n[a]);
    if (n[a] / d->ds[a] < 2)
      return fail(MH3D_ERR_INVALID, "decimated axis %d has fewer than 2 samples", a);
  }
  if (flat && !d->psf)
    return fail(MH3D_ERR_INVALID, "a 2D grid (ny = 1) takes user PSFs (the analytic PSF is the 3D one)");
  if (d->nz % 2) return fail(MH3D_ERR_INVALID, "nz must be even");
  if ((d->nz / d->ds[2]) % 2) return fail(MH3D_ERR_INVALID, "nz/ds[2] must be even");
  if (!(d->voxel_mm > 0)) return fail(MH3D_ERR_INVALID, "voxel_mm must be > 0");
  if (d->n_harm < 1 || d->n_harm > 32) return fail(MH3D_ERR_INVALID, "n_harm must be in [1, 32]");
  if (!d->harm) return fail(MH3D_ERR_INVALID, "harm is NULL");
  for (int i = 0; i < d->n_harm; ++i) {
    if (d->harm[i] < 2) return fail(MH3D_ERR_INVALID, "harmonic %d < 2", d->harm[i]);
    // the analytic PSF is defined by k; user PSFs only label their portraits (several
    // scans may repeat a harmonic)
    if (!d->psf && i && d->harm[i] <= d->harm[i - 1])
      return fail(MH3D_ERR_INVALID, "harmonics must increase strictly (analytic PSF)");
    if (d->harm[i] + d->order_offset < 1 || d->harm[i] + d->order_offset > 24)
      return fail(MH3D_ERR_INVALID, "derivative order k + order_offset must be in [1, 24]");
  }
  if (!d->psf && !(d->a_per_mm > 0)) return fail(MH3D_ERR_INVALID, "a_per_mm must be > 0");
  if (d->ncomp < 0 || d->ncomp > 3) return fail(MH3D_ERR_INVALID, "ncomp must be in [0, 3]");
  if (d->ncomp > 1 && (!d->psf || !d->sens))
    return fail(MH3D_ERR_INVALID, "the vector model (ncomp > 1) needs user PSFs and sensitivities");
  if (!d->sens)
    for (int a = 0; a < 3; ++a)
      if (!(d->sigma_mm[a] > 0)) return fail(MH3D_ERR_INVALID, "sigma_mm[%d] must be > 0", a);
  if (!(d->lambda >= 0)) return fail(MH3D_ERR_INVALID, "lambda must be >= 0");
  if (d->reg_kind != 0 && d->reg_kind != 1) return fail(MH3D_ERR_INVALID, "reg_kind must be 0 or 1");
  if (!(d->alpha >= 0.0) || !(d->alpha < 1e30)) return fail(MH3D_ERR_INVALID, "alpha must be finite and >= 0");
  if (d->alpha > 0.0) {
    const int mn = std::min(d->nx, flat ? d->nz : std::min(d->ny, d->nz));
    if (d->alpha_width < 1 || 2 * d->alpha_width > mn)
      return fail(MH3D_ERR_INVALID, "alpha_width must be in [1, min(nx, ny, nz)/2] when alpha > 0");
  } else if (d->alpha_width != 0) {
    return fail(MH3D_ERR_INVALID, "alpha_width must be 0 when alpha = 0");
  }
  for (int a = 0; a < 3; ++a) {
    if (d->pad[a] < 0 || d->pad[a] % d->ds[a])
      return fail(MH3D_ERR_INVALID, "pad[%d] = %d must be a non-negative multiple of ds[%d]", a, d->pad[a], a);
    if (!(a == 1 && flat) && (n[a] - 2 * d->pad[a]) / d->ds[a] < 2)
      return fail(MH3D_ERR_INVALID, "the field of view along axis %d has fewer than 2 decimated samples", a);
  }

  memset(&g, 0, sizeof g);
  g.nx = d->nx; g.ny = d->ny; g.nz = d->nz; g.nzh = g.nz / 2 + 1;
  g.sx = d->ds[0]; g.sy = d->ds[1]; g.sz = d->ds[2];
  g.mx = g.nx / g.sx; g.my = g.ny / g.sy; g.mz = g.nz / g.sz; g.mzh = g.mz / 2 + 1;
  g.S = g.sx * g.sy * g.sz;
  g.nmem = g.sy * g.sz;
  g.ncls = g.my * g.mzh;
  g.plane = g.ncls * g.nmem;
  g.K = d->n_harm;
  g.npairs = (g.ny + 1) / 2;
  g.N = (long long)g.nx * g.ny * g.nz;
  g.M = (long long)g.mx * g.my * g.mz;
  g.C = d->ncomp > 1 ? d->ncomp : 1;
  g.padded = (d->pad[0] || d->pad[1] || d->pad[2]) ? 1 : 0;
  g.pxs = d->pad[0] / g.sx; g.pys = d->pad[1] / g.sy; g.pzs = d->pad[2] / g.sz;
  g.mxf = g.mx - 2 * g.pxs; g.myf = g.my - 2 * g.pys; g.mzf = g.mz - 2 * g.pzs;
  g.Mf = (long long)g.mxf * g.myf * g.mzf;
  g.hsz = (long long)g.plane * g.nx;
  g.lsy = pad_odd(g.ny);
  g.lsx = pad_odd(g.nx);
  g.lsmy = pad_odd(g.my);

  CHK(derive_tiles(g, L, tiles ? tiles->E : 0, tiles ? tiles->cpw : 0, tiles ? tiles->xb : 0, tiles ? tiles->ps : 0));

  // ---- plane kernels
  L.T_plane = 1024;
  L.lds_plane = sizeof(float2) * ((size_t)g.ny + g.nz + 2 * (size_t)plane_lds(g));
  // (+512 bytes: the block reduction of the step that the adjoint plane pass can run)
  if (L.lds_plane + 512 > kLdsLimit) return fail(MH3D_ERR_UNSUPPORTED, "x-plane of %dx%d does not fit in LDS", g.ny, g.nz);
  return MH3D_OK;
}

// ============================================================================ plan
enum { KID_PLANE_FWD = 0, KID_CLASS_FWD, KID_SMALL_INV, KID_SMALL_FWD, KID_CLASS_ADJ, KID_PLANE_ADJ, KID_AUX, KID_SOLVE_ITER,
       KID_UPDATE, KID_CLASS_NORMAL, KID_ADJ_AND_STORE };
static const char* kKernelNames[MH3D_NKERNEL] = {"plane_fwd", "class_fwd", "small_inv", "small_fwd", "class_adj",
                                                  "plane_adj", "aux", "solve_iter", "vol_update", "class_normal",
                                                  "adj_and_store"};

struct FastOps;

struct mh3d_plan_s {
  const FastOps* fast = nullptr;   // compile-time-geometry passes of the fused sequences (or none)
  bool fast_on = true;             // whether the fused sequences use them (mh3d_plan_path)
  bool each_batched = false;       // the single-harmonic descriptors have separate Q buffers
  mh3d_plan_desc desc;
  std::vector<int> harm;
  Geo g;
  Launch L;
  hipStream_t stream;          // caller's stream: every operation is ordered on it
  hipStream_t ls;              // stream kernels are enqueued on (the caller's)
  int compact;
  uint32_t imag_mask;
  uint32_t cmask[3];           // present (component, harmonic) PSF blocks, vector model
  // device memory
  void* hs = nullptr;          // spectra in class layout
  float* b = nullptr;          // sensitivity
  float2* uperm = nullptr;     // class-layout yz spectra of one volume (also adjoint V)
  float* sfs = nullptr;        // separable spectra (analytic PSF): x factors [K][nx]
  float2* set = nullptr;       // and the y-residue table [sy][my][nz/2 + 1]
  float2* G = nullptr;         // decimated spectra (forward)
  float2* Gp = nullptr;        // decimated spectra (adjoint)
  float* vol[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // rho[0], rho[1], y[0], y[1], u
  float2* tw32 = nullptr;
  double2* tw64 = nullptr;
  int off[6];                  // table offsets for nx, ny, nz, mx, my, mz
  double* prof = nullptr;      // [K][nx]
  double* env = nullptr;       // [ny][nz]
  double* partials = nullptr;
  double* hist = nullptr;      // solver history (device), capacity hist_cap
  int hist_cap = 0;
  DevState* st = nullptr;      // solver / power state
  VolDesc vdh;                 // host copy of the descriptor
  // device descriptors: [0] for the operator calls, [1] for the solver's passes
  // (mh3d_normal, mh3d_power_iteration, mh3d_solve), which split each x-plane over
  // ps_solve workgroups; vdu holds what was last uploaded
  VolDesc* vdd = nullptr;
  VolDesc vdu[2];
  int ps_solve = 0;
  VolDesc* vda = nullptr;      // the descriptor the current call's passes use, and its split
  int psa = 0;
  VolDesc* vdk = nullptr;      // device descriptors of the single harmonics (K of them)
  int batch_refs = 0;          // batches holding this plan (tiles are frozen while > 0)
  int pi_iters = 0;            // cached step-size estimate: power iterations (0: none), seed, L
  uint64_t pi_seed = 0;
  double pi_lmax = 0.0;
  size_t bytes = 0;
  // profiling
  bool prof_on = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> free_events;
  double ms[MH3D_NKERNEL];
  int64_t launches[MH3D_NKERNEL];
};

static mh3d_status dalloc(mh3d_plan_t p, void** ptr, size_t bytes) {
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    *ptr = nullptr;
    return fail(MH3D_ERR_OOM, "hipMalloc(%zu) failed", bytes);
  }
  p->bytes += bytes;
  return MH3D_OK;
}

static size_t plan_bytes(const Geo& g, bool compact) {
  size_t s = 0;
  s += (size_t)g.C * g.K * g.hsz * (compact ? 4 : 8);
  s += (size_t)g.C * g.N * 4;                         // b
  s += (size_t)g.C * g.nx * g.plane * 8;              // uperm
  s += 2 * (size_t)g.K * g.mx * g.ncls * 8;           // G, Gp
  s += 5 * (size_t)g.N * 4;                           // vol
  s += (size_t)(2 * (g.nx + g.ny + g.nz) + g.mx + g.my + g.mz) * 24;
  s += ((size_t)g.K * g.nx + (size_t)g.ny * g.nz) * 8;
  if (compact) s += (size_t)g.K * g.nx * 4 + (size_t)g.sy * g.my * g.nzh * 8;   // separable factors
  return s;
}

extern "C" mh3d_status mh3d_plan_describe(const mh3d_plan_desc* desc, size_t* device_bytes,
                                          int64_t* n_volume, int64_t* n_portrait) {
  Geo g;
  Launch L;
  mh3d_status s = build_geo(desc, g, L);
  if (s != MH3D_OK) return s;
  if (device_bytes) *device_bytes = plan_bytes(g, desc->psf == nullptr);
  if (n_volume) *n_volume = g.N;
  if (n_portrait) *n_portrait = (int64_t)g.K * g.Mf;
  return MH3D_OK;
}

// ---------------------------------------------------------------------------- profiling helpers
static void drain_events(mh3d_plan_t p) {
  for (auto& e : p->pending) {
    float ms = 0.f;
    (void)hipEventSynchronize(e.second.second);
    (void)hipEventElapsedTime(&ms, e.second.first, e.second.second);
    p->ms[e.first] += ms;
    p->launches[e.first] += 1;
    p->free_events.push_back(e.second.first);
    p->free_events.push_back(e.second.second);
  }
  p->pending.clear();
}

struct Timer {
  mh3d_plan_t p;
  int kid;
  hipEvent_t a = nullptr, b = nullptr;
  Timer(mh3d_plan_t p_, int kid_) : p(p_), kid(kid_) {
    if (!p->prof_on) return;
    if (p->free_events.size() >= 2) {
      a = p->free_events.back(); p->free_events.pop_back();
      b = p->free_events.back(); p->free_events.pop_back();
    } else {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
    }
    (void)hipEventRecord(a, p->ls);
  }
  ~Timer() {
    if (!a) return;
    (void)hipEventRecord(b, p->ls);
    p->pending.push_back({kid, {a, b}});
    if (p->pending.size() > 4096) drain_events(p);
  }
};

// ---------------------------------------------------------------------------- fast passes
// Launchers of the compile-time-geometry passes (fast.hpp) of one grid, decimation and
// tile shape.  All passes of a fused sequence come from one entry (their slot layout is
// their own).
struct FastOps {
  int nx, ny, nz, sx, sy, sz, kmax;
  int nbp, ncls_blocks, tc;
  size_t lds_plane, lds_class;
  void (*plane_fwd)(hipStream_t, const VolDesc*, int src, const float* a);
  void (*cls)(hipStream_t, const VolDesc*, int mode, int chk);
  void (*plane_adj)(hipStream_t, const VolDesc*, int out, AdjOut ao);
  void (*adj_and_store)(hipStream_t, const VolDesc*, AdjOut ao, float* d, int nsmall, int xb);
  void (*small_inv)(hipStream_t, const VolDesc*, float* d, int nsmall, int xb);
  // A^T of nv single-harmonic descriptors at once (each with its own qx): out volumes
  // out + v N for v < nv
  void (*adjoint_each)(hipStream_t, const VolDesc*, int nv, float* out);
  // the portraits' small-grid spectra into G' (as k_small_fwd)
  void (*small_fwd)(hipStream_t, const VolDesc*, const float* r, float2* out, int nsmall, int xb);
};

template <class G>
struct FastImpl {
  static void plane_fwd(hipStream_t s, const VolDesc* vd, int src, const float* a) {
    const dim3 grid(G::NBP), block(G::TPF);
    switch (src) {
      case SRC_PLAIN: k_fast_plane_fwd<G, SRC_PLAIN><<<grid, block, G::LDS_PLANE, s>>>(vd, a); break;
      case SRC_FISTA_Y: k_fast_plane_fwd<G, SRC_FISTA_Y><<<grid, block, G::LDS_PLANE, s>>>(vd, a); break;
      default: k_fast_plane_fwd<G, SRC_SCALED><<<grid, block, G::LDS_PLANE, s>>>(vd, a); break;
    }
  }
  static void cls(hipStream_t s, const VolDesc* vd, int mode, int chk) {
    const dim3 grid(G::NCLS / G::CPC), block(G::TC);
    switch (mode) {
      case NRM_RESID: k_fast_col<G, NRM_RESID><<<grid, block, G::LDS_COL, s>>>(vd, chk); break;
      case NRM_PLAIN: k_fast_col<G, NRM_PLAIN><<<grid, block, G::LDS_COL, s>>>(vd, chk); break;
      case COL_FWD: k_fast_col<G, COL_FWD><<<grid, block, G::LDS_COL, s>>>(vd, chk); break;
      case COL_ADJ: k_fast_col<G, COL_ADJ><<<grid, block, G::LDS_COL, s>>>(vd, chk); break;
      default: k_fast_col<G, NRM_STORE><<<grid, block, G::LDS_COL, s>>>(vd, chk); break;
    }
  }
  static void plane_adj(hipStream_t s, const VolDesc* vd, int out, AdjOut ao) {
    const dim3 grid(G::NBP), block(G::TP);
    if (out == OUT_STEP_NORMAL) k_fast_plane_adj<G, OUT_STEP_NORMAL><<<grid, block, G::LDS_PLANE, s>>>(vd, ao);
    else if (out == OUT_STEP_FISTA) k_fast_plane_adj<G, OUT_STEP_FISTA><<<grid, block, G::LDS_PLANE, s>>>(vd, ao);
    else k_fast_plane_adj<G, OUT_SCALE_B><<<grid, block, G::LDS_PLANE, s>>>(vd, ao);
  }
  static void adj_and_store(hipStream_t s, const VolDesc* vd, AdjOut ao, float* d, int nsmall, int xb) {
    k_fast_adj_and_store<G><<<dim3(G::NBP + nsmall), dim3(G::TP), std::max(G::small_lds(xb), G::LDS_PLANE), s>>>(
        vd, ao, d);
  }
  static void small_inv(hipStream_t s, const VolDesc* vd, float* d, int nsmall, int xb) {
    k_fast_small_inv<G><<<dim3(nsmall), dim3(G::TP), G::small_lds(xb), s>>>(vd, d);
  }
  static void small_fwd(hipStream_t s, const VolDesc* vd, const float* r, float2* out, int nsmall, int xb) {
    k_fast_small_fwd<G><<<dim3(nsmall), dim3(G::TP), G::small_lds(xb), s>>>(vd, r, out);
  }
  static void adjoint_each(hipStream_t s, const VolDesc* vd, int nv, float* out) {
    k_fast_col<G, COL_ADJ><<<dim3(G::NCLS / G::CPC, nv), dim3(G::TC), G::LDS_COL, s>>>(vd, 0);
    AdjOut ao;
    ao.out = out;
    ao.yin = nullptr;
    k_fast_plane_adj<G, OUT_SCALE_B><<<dim3(G::NBP, nv), dim3(G::TP), G::LDS_PLANE, s>>>(vd, ao);
  }
  static FastOps ops() {
    return FastOps{G::NX, G::NY, G::NZ, G::SX, G::SY, G::SZ, G::KMAX, G::NBP, G::NCLS / G::CPC, G::TC,
                   G::LDS_PLANE, G::LDS_COL, &plane_fwd, &cls, &plane_adj, &adj_and_store, &small_inv,
                   &adjoint_each, &small_fwd};
  }
};

// Grids with compile-time passes: (nx, ny, nz, sx, sy, sz, columns per column-pass block,
// largest harmonic count).
static const FastOps kFast[] = {
    FastImpl<FastGeo<128, 128, 128, 2, 4, 4, 4, 12, 512, 512, 134>>::ops(),   // 128^3, k = 2..12
    FastImpl<FastGeo<96, 96, 64, 2, 2, 2, 4, 8, 512, 512>>::ops(),            // 96 x 96 x 64, k = 2..8
    // small grids of the parity tests: every y split (1 to 4), radix 3 along x and y
    FastImpl<FastGeo<32, 32, 32, 2, 4, 4, 4, 12>>::ops(),
    FastImpl<FastGeo<16, 24, 16, 2, 2, 2, 4, 8>>::ops(),
    FastImpl<FastGeo<16, 16, 16, 2, 1, 2, 4, 8>>::ops(),
    FastImpl<FastGeo<24, 24, 16, 2, 3, 2, 4, 8>>::ops(),
};

// The entry serving plan p (scalar model, analytic spectra, no padding), or NULL.  Its
// intermediates (sy shares and one more of nx * columns) live in the class-layout
// buffer, which holds nx * columns * sy * sz values.
static const FastOps* find_fast(const Geo& g, bool compact) {
  if (!compact || g.C != 1 || g.padded) return nullptr;
  if (g.sy + 1 > g.nmem) return nullptr;
  for (const FastOps& f : kFast)
    if (f.nx == g.nx && f.ny == g.ny && f.nz == g.nz && f.sx == g.sx && f.sy == g.sy && f.sz == g.sz && g.K <= f.kmax)
      return &f;
  return nullptr;
}

static mh3d_status last_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MH3D_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return MH3D_OK;
}

// ---------------------------------------------------------------------------- single-volume launchers
static mh3d_status launch_plane_fwd(mh3d_plan_t p, int src, const float* a) {
  Timer t(p, KID_PLANE_FWD);
  // vector model: one group of ps * nx blocks per component (a raw source has one)
  dim3 grid((src == SRC_RAW ? 1 : p->g.C) * p->psa * p->g.nx), block(p->L.T_plane);
  const size_t lds = p->L.lds_plane;
  switch (src) {
    case SRC_PLAIN: k_plane_fwd<SRC_PLAIN><<<grid, block, lds, p->ls>>>(p->vda, nullptr, a); break;
    case SRC_RAW: k_plane_fwd<SRC_RAW><<<grid, block, lds, p->ls>>>(p->vda, nullptr, a); break;
    case SRC_FISTA_Y: k_plane_fwd<SRC_FISTA_Y><<<grid, block, lds, p->ls>>>(p->vda, nullptr, a); break;
    default: k_plane_fwd<SRC_SCALED><<<grid, block, lds, p->ls>>>(p->vda, nullptr, a); break;
  }
  return last_launch("k_plane_fwd");
}

// HC: 0 compact (analytic) spectra, 1 complex (user) spectra, 2 complex spectra of a
// vector-model plan (components looped inside the class passes).
template <int HC, int E>
static void class_fwd_t(mh3d_plan_t p, int chk, const VolDesc* vd, int mode) {
  k_class_fwd<HC == 0 ? 0 : 1, E, HC == 2>
      <<<dim3(p->g.ncls / p->g.cpw), dim3(p->L.T_class), p->L.lds_class, p->ls>>>(vd, chk, mode);
}
template <int HC, int E>
static void class_adj_t(mh3d_plan_t p, int chk, const VolDesc* vd, int) {
  k_class_adj<HC == 0 ? 0 : 1, E, HC == 2>
      <<<dim3(p->g.ncls / p->g.cpw), dim3(p->L.T_class), p->L.lds_class, p->ls>>>(vd, chk);
}

#define E_DISPATCH(HCV, FN)                             \
  switch (p->g.E) {                                     \
    case 9: FN<HCV, 9>(p, chk, vd, mode); break;        \
    case 8: FN<HCV, 8>(p, chk, vd, mode); break;        \
    case 6: FN<HCV, 6>(p, chk, vd, mode); break;        \
    case 4: FN<HCV, 4>(p, chk, vd, mode); break;        \
    case 3: FN<HCV, 3>(p, chk, vd, mode); break;        \
    case 2: FN<HCV, 2>(p, chk, vd, mode); break;        \
    default: FN<HCV, 1>(p, chk, vd, mode); break;       \
  }

// mode: FWD_G, FWD_ADJ, FWD_G_AND_ADJ or FWD_RESID (where the decimated spectra go).
static mh3d_status launch_class_fwd(mh3d_plan_t p, int chk, int mode) {
  Timer t(p, KID_CLASS_FWD);
  const VolDesc* vd = p->vda;
  if (p->compact) { E_DISPATCH(0, class_fwd_t) } else if (p->g.C > 1) { E_DISPATCH(2, class_fwd_t) } else { E_DISPATCH(1, class_fwd_t) }
  return last_launch("k_class_fwd");
}
// vd: a single-harmonic descriptor (per-harmonic back-projection) or NULL for the plan's.
static mh3d_status launch_class_adj(mh3d_plan_t p, int chk, const VolDesc* vd = nullptr) {
  Timer t(p, KID_CLASS_ADJ);
  if (!vd) vd = p->vda;
  const int mode = 0;
  if (p->compact) { E_DISPATCH(0, class_adj_t) } else if (p->g.C > 1) { E_DISPATCH(2, class_adj_t) } else { E_DISPATCH(1, class_adj_t) }
  return last_launch("k_class_adj");
}

// Scalar plans without boundary padding run the forward and adjoint class passes of the
// normal operator, the solver's updates and A then A^T as one (k_class_normal).
static bool fused_class(mh3d_plan_t p) { return p->g.C == 1 && !p->g.padded; }

template <int HC, int E>
static void class_normal_t(mh3d_plan_t p, int chk, const VolDesc* vd, int mode) {
  k_class_normal<HC, E><<<dim3(p->g.ncls / p->g.cpw), dim3(p->L.T_class), p->L.lds_class, p->ls>>>(vd, chk, mode);
}
// mode: NRM_RESID, NRM_PLAIN or NRM_STORE.
static mh3d_status launch_class_normal(mh3d_plan_t p, int chk, int mode) {
  Timer t(p, KID_CLASS_NORMAL);
  const VolDesc* vd = p->vda;
  if (p->compact) { E_DISPATCH(0, class_normal_t) } else { E_DISPATCH(1, class_normal_t) }
  return last_launch("k_class_normal");
}

static mh3d_status launch_small_inv(mh3d_plan_t p, int epi, float* d) {
  Timer t(p, KID_SMALL_INV);
  dim3 grid(p->g.K * (p->g.mx / p->g.xb)), block(p->L.T_small);
  const size_t lds = p->L.lds_small;
  switch (epi) {
    case EPI_STORE: k_small_inv<EPI_STORE><<<grid, block, lds, p->ls>>>(p->vda, nullptr, d); break;
    case EPI_RESID_BACK: k_small_inv<EPI_RESID_BACK><<<grid, block, lds, p->ls>>>(p->vda, nullptr, d); break;
    case EPI_STORE_BACK: k_small_inv<EPI_STORE_BACK><<<grid, block, lds, p->ls>>>(p->vda, nullptr, d); break;
    default: k_small_inv<EPI_BACK><<<grid, block, lds, p->ls>>>(p->vda, nullptr, d); break;
  }
  return last_launch("k_small_inv");
}

// out: destination of the spectra (NULL: G', the adjoint's input).
static mh3d_status launch_small_fwd(mh3d_plan_t p, const float* r, float2* out = nullptr) {
  Timer t(p, KID_SMALL_FWD);
  k_small_fwd<<<dim3(p->g.K * (p->g.mx / p->g.xb)), dim3(p->L.T_small), p->L.lds_small, p->ls>>>(p->vda, r, out);
  return last_launch("k_small_fwd");
}
static bool use_fast(mh3d_plan_t p);
// The portraits' small-grid spectra into G' for A^T alone and the back-projections: the
// compile-time pass where the plan runs those passes
static mh3d_status launch_small_fwd_adj(mh3d_plan_t p, const float* r) {
  if (!use_fast(p)) return launch_small_fwd(p, r);
  Timer t(p, KID_SMALL_FWD);
  p->fast->small_fwd(p->ls, p->vda, r, p->Gp, p->g.K * (p->g.mx / p->g.xb), p->g.xb);
  return last_launch("k_fast_small_fwd");
}

static mh3d_status launch_plane_adj(mh3d_plan_t p, int out, float* o, const float* yin,
                                    const VolDesc* vd = nullptr) {
  Timer t(p, KID_PLANE_ADJ);
  if (!vd) vd = p->vda;
  dim3 grid(p->psa * p->g.nx), block(p->L.T_plane);
  const size_t lds = p->L.lds_plane;
  AdjOut ao;
  ao.out = o;
  ao.yin = yin;
  switch (out) {
    case OUT_SCALE_B: k_plane_adj<OUT_SCALE_B><<<grid, block, lds, p->ls>>>(vd, nullptr, ao); break;
    case OUT_STEP_NORMAL: k_plane_adj<OUT_STEP_NORMAL><<<grid, block, lds, p->ls>>>(vd, nullptr, ao); break;
    case OUT_STEP_FISTA: k_plane_adj<OUT_STEP_FISTA><<<grid, block, lds, p->ls>>>(vd, nullptr, ao); break;
    default: k_plane_adj<OUT_U><<<grid, block, lds, p->ls>>>(vd, nullptr, ao); break;
  }
  return last_launch("k_plane_adj");
}

// After the fused class pass of A then A^T: the adjoint plane pass (x = A^T d) and the
// small-grid inverse pass that writes d, as one launch of ps nx + K mx/xb blocks.
static mh3d_status launch_adj_and_store(mh3d_plan_t p, float* d, float* x) {
  Timer t(p, KID_ADJ_AND_STORE);
  AdjOut ao;
  ao.out = x;
  ao.yin = nullptr;
  const dim3 grid(p->psa * p->g.nx + p->g.K * (p->g.mx / p->g.xb)), block(p->L.T_merge);
  k_adj_and_store<<<grid, block, std::max(p->L.lds_plane, p->L.lds_small), p->ls>>>(p->vda, ao, d);
  return last_launch("k_adj_and_store");
}

// The fused sequences run the compile-time passes of fast.hpp when the plan has them.
static bool use_fast(mh3d_plan_t p) {
  // the compile-time small-grid pass takes x'-blocks of 1, 2, 4 or 8 planes
  const int xb = p->g.xb;
  return p->fast && p->fast_on && (xb == 1 || xb == 2 || xb == 4 || xb == 8);
}

// Scalar plans with one workgroup per x-plane also run the next update's forward plane
// pass in the launch of the step (k_step_and_fwd).
static bool step_and_fwd(mh3d_plan_t p) { return p->g.C == 1 && p->psa == 1 && !use_fast(p); }

// ---- the fused sequences on the compile-time passes
static mh3d_status fast_plane_fwd(mh3d_plan_t p, int src, const float* a) {
  Timer t(p, KID_PLANE_FWD);
  p->fast->plane_fwd(p->ls, p->vda, src, a);
  return last_launch("k_fast_plane_fwd");
}
static mh3d_status fast_class(mh3d_plan_t p, int chk, int mode) {
  Timer t(p, KID_CLASS_NORMAL);
  p->fast->cls(p->ls, p->vda, mode, chk);
  return last_launch("k_fast_class");
}
static mh3d_status fast_adj_and_store(mh3d_plan_t p, float* d, float* x) {
  Timer t(p, KID_ADJ_AND_STORE);
  AdjOut ao;
  ao.out = x;
  ao.yin = nullptr;
  p->fast->adj_and_store(p->ls, p->vda, ao, d, p->g.K * (p->g.mx / p->g.xb), p->g.xb);
  return last_launch("k_fast_adj_and_store");
}
static mh3d_status fast_class_alone(mh3d_plan_t p, int mode) {
  Timer t(p, mode == COL_FWD ? KID_CLASS_FWD : KID_CLASS_ADJ);
  p->fast->cls(p->ls, p->vda, mode, 0);
  return last_launch("k_fast_col");
}
static mh3d_status fast_small_inv(mh3d_plan_t p, float* d) {
  Timer t(p, KID_SMALL_INV);
  p->fast->small_inv(p->ls, p->vda, d, p->g.K * (p->g.mx / p->g.xb), p->g.xb);
  return last_launch("k_fast_small_inv");
}
static mh3d_status fast_plane_adj_out(mh3d_plan_t p, float* x) {
  Timer t(p, KID_PLANE_ADJ);
  AdjOut ao;
  ao.out = x;
  ao.yin = nullptr;
  p->fast->plane_adj(p->ls, p->vda, OUT_SCALE_B, ao);
  return last_launch("k_fast_plane_adj");
}
// the adjoint plane pass that ends a step (UPD_NORMAL: out, w = yin; UPD_FISTA), then the
// one-block finish of its FP64 sums
static mh3d_status fast_adjoint_step(mh3d_plan_t p, int upd, float* o, const float* yin) {
  AdjOut ao;
  ao.out = o;
  ao.yin = yin;
  {
    Timer t(p, KID_PLANE_ADJ);
    p->fast->plane_adj(p->ls, p->vda, upd == UPD_NORMAL ? OUT_STEP_NORMAL : OUT_STEP_FISTA, ao);
    CHK(last_launch("k_fast_plane_adj"));
  }
  Timer t(p, KID_UPDATE);
  if (upd == UPD_NORMAL) k_vol_finish<UPD_NORMAL><<<1, 256, 0, p->ls>>>(p->vda, nullptr);
  else k_vol_finish<UPD_FISTA><<<1, 256, 0, p->ls>>>(p->vda, nullptr);
  return last_launch("k_vol_finish");
}

static mh3d_status launch_step_and_fwd(mh3d_plan_t p) {
  {
    Timer t(p, KID_PLANE_ADJ);
    AdjOut ao;
    ao.out = nullptr;
    ao.yin = nullptr;
    k_step_and_fwd<<<dim3(p->g.nx), dim3(p->L.T_plane), p->L.lds_plane, p->ls>>>(p->vda, nullptr, ao);
    CHK(last_launch("k_step_and_fwd"));
  }
  Timer t(p, KID_UPDATE);
  k_vol_finish<UPD_FISTA><<<1, 256, 0, p->ls>>>(p->vda, nullptr);
  return last_launch("k_vol_finish");
}

// Scalar plans finish a solver step inside the adjoint plane pass (its u = b . v stays
// in registers); vector plans, whose plane pass sums the components, run the update
// pass after it.  The block count of the step's FP64 sums is the descriptor's nb_upd.
static bool step_in_plane_pass(mh3d_plan_t p) { return p->g.C == 1; }

// The adjoint plane pass and the rest of a solver step: out = (A^T A + lambda T^T T)(s w)
// (UPD_NORMAL, w = yin) or one accelerated projected gradient update (UPD_FISTA).
static mh3d_status launch_adjoint_step(mh3d_plan_t p, int upd, float* o, const float* yin) {
  if (step_in_plane_pass(p)) {
    CHK(launch_plane_adj(p, upd == UPD_NORMAL ? OUT_STEP_NORMAL : OUT_STEP_FISTA, o, yin));
  } else {
    CHK(launch_plane_adj(p, OUT_U, nullptr, nullptr));
  }
  Timer t(p, KID_UPDATE);
  AdjOut ao;
  ao.out = o;
  ao.yin = yin;
  const dim3 grid(update_blocks(p->g.N)), block(UPD_THREADS);
  if (upd == UPD_NORMAL) {
    if (!step_in_plane_pass(p)) k_vol_update<UPD_NORMAL><<<grid, block, 0, p->ls>>>(p->vda, nullptr, ao);
    k_vol_finish<UPD_NORMAL><<<1, 256, 0, p->ls>>>(p->vda, nullptr);
  } else {
    if (!step_in_plane_pass(p)) k_vol_update<UPD_FISTA><<<grid, block, 0, p->ls>>>(p->vda, nullptr, ao);
    k_vol_finish<UPD_FISTA><<<1, 256, 0, p->ls>>>(p->vda, nullptr);
  }
  return last_launch("k_vol_update / k_vol_finish");
}

// ---------------------------------------------------------------------------- state
__global__ void k_state_set(DevState* st, DevState v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st = v;
}

static mh3d_status state_set(mh3d_plan_t p, const DevState& v) {
  Timer t(p, KID_AUX);
  hipLaunchKernelGGL(k_state_set, dim3(1), dim3(64), 0, p->ls, p->st, v);
  return last_launch("k_state_set");
}

static mh3d_status upload_desc(mh3d_plan_t p) {
  p->vdu[0] = p->vdh;
  p->vdu[1] = p->vdh;
  p->vdu[1].g.ps = p->ps_solve;
  p->vdu[1].nb_upd = use_fast(p) ? p->fast->nbp : (p->g.C == 1 ? p->ps_solve * p->g.nx : update_blocks(p->g.N));
  HIPCHK(hipMemcpyAsync(p->vdd, p->vdu, sizeof p->vdu, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return MH3D_OK;
}

// Runs the enclosing call's passes with the solver's plane split (descriptor [1]).
struct SolverPasses {
  mh3d_plan_t p;
  VolDesc* vda;
  int psa;
  explicit SolverPasses(mh3d_plan_t q) : p(q), vda(q->vda), psa(q->psa) {
    p->vda = p->vdd + 1;
    p->psa = p->ps_solve;
  }
  ~SolverPasses() {
    p->vda = vda;
    p->psa = psa;
  }
};

// Two timing events destroyed on every exit path of the call that created them.
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair() = default;
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
  hipError_t create() {
    hipError_t r = hipEventCreate(&e0);
    return r != hipSuccess ? r : hipEventCreate(&e1);
  }
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// ---------------------------------------------------------------------------- plan build
static mh3d_status build_tables(mh3d_plan_t p) {
  const Geo& g = p->g;
  const int lens[6] = {g.nx, g.ny, g.nz, g.mx, g.my, g.mz};
  int total = 0;
  for (int i = 0; i < 6; ++i) { p->off[i] = total; total += lens[i]; }
  CHK(dalloc(p, (void**)&p->tw32, sizeof(float2) * total));
  CHK(dalloc(p, (void**)&p->tw64, sizeof(double2) * total));
  for (int i = 0; i < 6; ++i) {
    hipLaunchKernelGGL(k_twiddles, dim3(1), dim3(256), 0, p->stream, lens[i], p->tw32 + p->off[i], p->tw64 + p->off[i]);
    CHK(last_launch("k_twiddles"));
  }
  return MH3D_OK;
}

static mh3d_status build_spectra_analytic(mh3d_plan_t p) {
  const Geo& g = p->g;
  const mh3d_plan_desc& d = p->desc;
  std::vector<int> order(g.K);
  p->imag_mask = 0;
  for (int k = 0; k < g.K; ++k) {
    order[k] = p->harm[k] + d.order_offset;
    if (order[k] % 2 == 0) p->imag_mask |= (1u << k);   // odd profile -> imaginary spectrum
  }
  int* d_order = nullptr;
  double2 *fhat = nullptr, *tmp = nullptr, *ehat = nullptr;
  double *fn2 = nullptr, *rows = nullptr, *scale = nullptr;
  size_t keep = p->bytes;
  CHK(dalloc(p, (void**)&d_order, sizeof(int) * g.K));
  CHK(dalloc(p, (void**)&fhat, sizeof(double2) * g.K * g.nx));
  CHK(dalloc(p, (void**)&tmp, sizeof(double2) * g.ny * g.nz));
  CHK(dalloc(p, (void**)&ehat, sizeof(double2) * g.ny * g.nzh));
  CHK(dalloc(p, (void**)&fn2, sizeof(double) * g.K));
  CHK(dalloc(p, (void**)&rows, sizeof(double) * g.ny));
  CHK(dalloc(p, (void**)&scale, sizeof(double) * g.K));
  HIPCHK(hipMemcpyAsync(d_order, order.data(), sizeof(int) * g.K, hipMemcpyHostToDevice, p->stream));
  const int T = 256;
  hipLaunchKernelGGL(k_psf_profile, dim3(g.K), dim3(T), sizeof(double2) * 3 * g.nx, p->stream, g.nx, d_order,
                     d.a_per_mm * d.voxel_mm, p->tw64 + p->off[0], p->prof, fhat, fn2);
  CHK(last_launch("k_psf_profile"));
  hipLaunchKernelGGL(k_psf_env_rows, dim3(g.ny), dim3(T), sizeof(double2) * 3 * g.nz, p->stream, g.ny, g.nz,
                     d.a_per_mm, d.voxel_mm, p->tw64 + p->off[2], p->env, tmp, rows);
  CHK(last_launch("k_psf_env_rows"));
  hipLaunchKernelGGL(k_psf_env_cols, dim3(g.nzh), dim3(T), sizeof(double2) * 3 * g.ny, p->stream, g.ny, g.nz,
                     p->tw64 + p->off[1], tmp, ehat);
  CHK(last_launch("k_psf_env_cols"));
  hipLaunchKernelGGL(k_psf_scales, dim3(1), dim3(64), 0, p->stream, g.K, g.ny, g.N, fn2, rows, scale);
  CHK(last_launch("k_psf_scales"));
  hipLaunchKernelGGL(k_psf_assemble, dim3(2048), dim3(256), 0, p->stream, g, fhat, ehat, scale, p->imag_mask, 1, p->hs);
  CHK(last_launch("k_psf_assemble"));
  hipLaunchKernelGGL(k_sep_tables, dim3(64), dim3(256), 0, p->stream, g, fhat, ehat, scale, p->imag_mask,
                     p->tw64 + p->off[1], p->sfs, p->set);
  CHK(last_launch("k_sep_tables"));
  HIPCHK(hipStreamSynchronize(p->stream));
  (void)hipFree(d_order); (void)hipFree(fhat); (void)hipFree(tmp); (void)hipFree(ehat);
  (void)hipFree(fn2); (void)hipFree(rows); (void)hipFree(scale);
  p->bytes = keep;
  return MH3D_OK;
}

// Vector model: which (component, harmonic) PSF blocks are not identically zero.  The
// class passes skip the others (their products are zero).  A harmonic with no nonzero
// block keeps component 0.
static mh3d_status component_masks(mh3d_plan_t p) {
  const Geo& g = p->g;
  const uint32_t all = g.K >= 32 ? ~0u : ((1u << g.K) - 1u);
  for (int c = 0; c < 3; ++c) p->cmask[c] = c < g.C ? all : 0u;
  if (g.C == 1) return MH3D_OK;
  const int nb = g.C * g.K, ns = 64;
  int* d_flags = nullptr;
  HIPCHK(hipMalloc(&d_flags, sizeof(int) * nb * ns));
  k_nonzero_blocks<<<dim3(nb, ns), dim3(256), 0, p->stream>>>(p->desc.psf, g.N, d_flags);
  mh3d_status s = last_launch("k_nonzero_blocks");
  std::vector<int> f((size_t)nb * ns, 1);
  if (s == MH3D_OK && (hipMemcpyAsync(f.data(), d_flags, sizeof(int) * nb * ns, hipMemcpyDeviceToHost, p->stream) !=
                           hipSuccess ||
                       hipStreamSynchronize(p->stream) != hipSuccess))
    s = fail(MH3D_ERR_HIP, "reading the PSF block flags failed");
  (void)hipFree(d_flags);
  if (s != MH3D_OK) return s;
  for (int c = 0; c < g.C; ++c)
    for (int k = 0; k < g.K; ++k) {
      int any = 0;
      for (int q = 0; q < ns; ++q) any |= f[(size_t)(c * g.K + k) * ns + q];
      if (!any) p->cmask[c] &= ~(1u << k);
    }
  const uint32_t some = p->cmask[0] | p->cmask[1] | p->cmask[2];
  p->cmask[0] |= all & ~some;
  return MH3D_OK;
}

static mh3d_status build_spectra_user(mh3d_plan_t p) {
  const Geo& g = p->g;
  p->imag_mask = 0;
  size_t lds = sizeof(float2) * ((size_t)g.nx + 2 * (size_t)g.lsx * g.cpw * g.nmem);
  // component i's spectra follow component i - 1's (vector model)
  for (int k = 0; k < g.C * g.K; ++k) {
    CHK(launch_plane_fwd(p, SRC_RAW, p->desc.psf + (long long)k * g.N));
    k_class_hcopy<<<dim3(g.ncls / g.cpw), dim3(p->L.T_class), lds, p->ls>>>(g, k, p->uperm,
                         reinterpret_cast<float2*>(p->hs), p->tw32 + p->off[0]);
    CHK(last_launch("k_class_hcopy"));
  }
  return MH3D_OK;
}

extern "C" void mh3d_destroy(mh3d_plan_t p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (auto& e : p->pending) { (void)hipEventDestroy(e.second.first); (void)hipEventDestroy(e.second.second); }
  for (auto e : p->free_events) (void)hipEventDestroy(e);
  void* bufs[] = {p->hs, p->b, p->uperm, p->G, p->Gp, p->vol[0], p->vol[1], p->vol[2], p->vol[3], p->vol[4],
                  p->tw32, p->tw64, p->prof, p->env, p->partials, p->st, p->vdd, p->vdk, p->hist, p->sfs, p->set};
  for (void* q : bufs)
    if (q) (void)hipFree(q);
  delete p;
}

static void fill_desc(mh3d_plan_t p) {
  VolDesc& v = p->vdh;
  memset(&v, 0, sizeof v);
  v.g = p->g;
  v.hs = p->hs;
  v.imag_mask = p->imag_mask;
  v.compact = p->compact;
  v.b = p->b;
  v.uperm = p->uperm;
  v.G = p->G;
  v.Gp = p->Gp;
  v.rho[0] = p->vol[0];
  v.rho[1] = p->vol[1];
  v.y[0] = p->vol[2];
  v.y[1] = p->vol[3];
  v.d = nullptr;
  v.tw = p->tw32;
  for (int i = 0; i < 6; ++i) v.off[i] = p->off[i];
  v.st = p->st;
  v.partials = p->partials;
  v.hist = p->hist;
  v.hist_len = 0;
  v.k_first = 1;
  v.reg_kind = p->desc.reg_kind;
  v.lam = (float)p->desc.lambda;
  v.alpha = (float)p->desc.alpha;
  v.aw = p->desc.alpha_width;
  v.T_class = p->L.T_class;
  v.u = p->vol[4];
  // blocks whose FP64 sums a step leaves: the adjoint plane pass's (scalar plans) or the
  // update pass's (vector plans)
  v.nb_upd = p->g.C == 1 ? p->g.ps * p->g.nx : update_blocks(p->g.N);
  v.ncomp = p->g.C;
  v.hs_cstride = (long long)p->g.K * p->g.hsz;
  v.sfs = p->sfs;
  v.set = p->set;
  v.cp = p->uperm;
  v.qx = p->uperm + (size_t)p->g.sy * p->g.nx * p->g.ncls;
  for (int c = 0; c < 3; ++c) v.cmask[c] = p->cmask[c];
}

// Descriptor of harmonic k alone: the same buffers with K = 1, the spectra and the
// decimated adjoint spectra offset to harmonic k.  The adjoint passes run with it
// give the harmonic's back-projection b (H_k^T P^T d_k) without the sum over k.
static mh3d_status upload_harmonic_descs(mh3d_plan_t p) {
  const Geo& g = p->g;
  std::vector<VolDesc> h(g.K, p->vdh);
  const size_t esz = p->compact ? sizeof(float) : sizeof(float2);
  // the compile-time passes: harmonic k's x factors, and its own Q buffer when the K of
  // them fit in the class-layout buffer (the column pass of A^T alone does not read the
  // shares that otherwise sit there), so the K adjoints run in one launch per pass
  const size_t nq = (size_t)g.nx * g.ncls;
  p->each_batched = p->fast && (size_t)g.K * nq <= (size_t)g.C * g.nx * g.plane;
  for (int k = 0; k < g.K; ++k) {
    h[k].g.K = 1;
    h[k].hs = (const char*)p->vdh.hs + (size_t)k * g.hsz * esz;
    h[k].Gp = p->vdh.Gp + (size_t)k * g.mx * g.ncls;
    h[k].imag_mask = (p->vdh.imag_mask >> k) & 1u;
    for (int c = 0; c < 3; ++c) h[k].cmask[c] = (p->vdh.cmask[c] >> k) & 1u;
    if (p->sfs) h[k].sfs = p->sfs + (size_t)k * g.nx;
    if (p->each_batched) h[k].qx = p->uperm + (size_t)k * nq;
  }
  HIPCHK(hipMemcpyAsync(p->vdk, h.data(), sizeof(VolDesc) * g.K, hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_plan(const mh3d_plan_desc* desc, mh3d_plan_t* out) {
  if (!out) return fail(MH3D_ERR_INVALID, "out is NULL");
  *out = nullptr;
  Geo g;
  Launch L;
  CHK(build_geo(desc, g, L));
  int dev_count = 0;
  if (hipGetDeviceCount(&dev_count) != hipSuccess || dev_count < 1)
    return fail(MH3D_ERR_HIP, "no HIP device available");
  mh3d_plan_t p = new mh3d_plan_s();
  p->desc = *desc;
  p->harm.assign(desc->harm, desc->harm + desc->n_harm);
  p->desc.harm = p->harm.data();
  p->g = g;
  p->L = L;
  p->stream = reinterpret_cast<hipStream_t>(desc->stream);
  p->ls = p->stream;
  p->compact = desc->psf ? 0 : 1;
  p->fast = find_fast(g, p->compact);
  memset(p->ms, 0, sizeof p->ms);
  memset(p->launches, 0, sizeof p->launches);
  auto bail = [&](mh3d_status s) { mh3d_destroy(p); return s; };
  mh3d_status s;
  const size_t hbytes = (size_t)g.C * g.K * g.hsz * (p->compact ? sizeof(float) : sizeof(float2));
  if ((s = dalloc(p, &p->hs, hbytes)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->b, sizeof(float) * g.C * g.N)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->uperm, sizeof(float2) * (size_t)g.C * g.nx * g.plane)) != MH3D_OK) return bail(s);
  if (p->compact) {
    if ((s = dalloc(p, (void**)&p->sfs, sizeof(float) * (size_t)g.K * g.nx)) != MH3D_OK) return bail(s);
    if ((s = dalloc(p, (void**)&p->set, sizeof(float2) * (size_t)g.sy * g.my * g.nzh)) != MH3D_OK) return bail(s);
  }
  if ((s = dalloc(p, (void**)&p->G, sizeof(float2) * (size_t)g.K * g.mx * g.ncls)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->Gp, sizeof(float2) * (size_t)g.K * g.mx * g.ncls)) != MH3D_OK) return bail(s);
  for (int i = 0; i < 5; ++i)
    if ((s = dalloc(p, (void**)&p->vol[i], sizeof(float) * g.N)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->prof, sizeof(double) * (size_t)g.K * g.nx)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->env, sizeof(double) * (size_t)g.ny * g.nz)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->partials, sizeof(double) * 4 * 1024)) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->st, sizeof(DevState))) != MH3D_OK) return bail(s);
  if ((s = dalloc(p, (void**)&p->vdd, 2 * sizeof(VolDesc))) != MH3D_OK) return bail(s);
  p->vda = p->vdd;
  p->psa = p->ps_solve = g.ps;
  if ((s = dalloc(p, (void**)&p->vdk, sizeof(VolDesc) * g.K)) != MH3D_OK) return bail(s);
  if ((s = build_tables(p)) != MH3D_OK) return bail(s);
  fill_desc(p);
  if ((s = upload_desc(p)) != MH3D_OK) return bail(s);
  if (desc->sens) {
    if (hipMemcpyAsync(p->b, desc->sens, sizeof(float) * g.C * g.N, hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
      return bail(fail(MH3D_ERR_HIP, "copy of the sensitivity map failed"));
  } else {
    hipLaunchKernelGGL(k_sensitivity, dim3(1024), dim3(256), 0, p->stream, g, desc->voxel_mm, desc->sigma_mm[0],
                       desc->sigma_mm[1], desc->sigma_mm[2], p->b);
    if ((s = last_launch("k_sensitivity")) != MH3D_OK) return bail(s);
  }
  DevState z;
  memset(&z, 0, sizeof z);
  if ((s = state_set(p, z)) != MH3D_OK) return bail(s);
  if (p->compact) s = build_spectra_analytic(p);
  else s = build_spectra_user(p);
  if (s == MH3D_OK) s = component_masks(p);
  if (s != MH3D_OK) return bail(s);
  fill_desc(p);   // imag_mask is known now
  if ((s = upload_desc(p)) != MH3D_OK) return bail(s);
  if ((s = upload_harmonic_descs(p)) != MH3D_OK) return bail(s);
  if (hipStreamSynchronize(p->stream) != hipSuccess) return bail(fail(MH3D_ERR_HIP, "plan build failed on the device"));
  *out = p;
  return MH3D_OK;
}

// ============================================================================ operators
static mh3d_status check_plan(mh3d_plan_t p) {
  if (!p) return fail(MH3D_ERR_INVALID, "plan is NULL");
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_forward_adjoint(mh3d_plan_t p, const float* rho, float* d, float* x) {
  CHK(check_plan(p));
  if (!rho || !d || !x) return fail(MH3D_ERR_INVALID, "NULL array");
  if (use_fast(p)) {
    CHK(fast_plane_fwd(p, SRC_PLAIN, rho));
    CHK(fast_class(p, 0, NRM_STORE));   // d's spectra and A^T's class pass
    return fast_adj_and_store(p, d, x);
  }
  if (fused_class(p)) {
    {
      // the forward plane pass has its launch to itself, as the solver's plane passes
      // do, so it takes their split; the adjoint plane blocks share their launch with
      // the small-grid blocks and keep the plan's
      SolverPasses sp(p);
      CHK(launch_plane_fwd(p, SRC_PLAIN, rho));
    }
    CHK(launch_class_normal(p, 0, NRM_STORE));   // d's spectra and A^T's class pass
    return launch_adj_and_store(p, d, x);
  }
  CHK(launch_plane_fwd(p, SRC_PLAIN, rho));
  if (p->g.padded) {
    CHK(launch_class_fwd(p, 0, FWD_G));
    CHK(launch_small_inv(p, EPI_STORE_BACK, d));   // stores d and starts A^T on its cropped copy
    CHK(launch_class_adj(p, 0));
  } else {
    CHK(launch_class_fwd(p, 0, FWD_G_AND_ADJ));    // A^T starts from d's spectra
    CHK(launch_small_inv(p, EPI_STORE, d));
    CHK(launch_class_adj(p, 0));
  }
  CHK(launch_plane_adj(p, OUT_SCALE_B, x, nullptr));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_forward(mh3d_plan_t p, const float* rho, float* d) {
  CHK(check_plan(p));
  if (!rho || !d) return fail(MH3D_ERR_INVALID, "NULL array");
  if (use_fast(p)) {
    CHK(fast_plane_fwd(p, SRC_PLAIN, rho));
    CHK(fast_class_alone(p, COL_FWD));
    return fast_small_inv(p, d);
  }
  CHK(launch_plane_fwd(p, SRC_PLAIN, rho));
  CHK(launch_class_fwd(p, 0, FWD_G));
  CHK(launch_small_inv(p, EPI_STORE, d));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_adjoint(mh3d_plan_t p, const float* d, float* rho) {
  CHK(check_plan(p));
  if (!rho || !d) return fail(MH3D_ERR_INVALID, "NULL array");
  if (use_fast(p)) {
    CHK(launch_small_fwd_adj(p, d));   // the portraits' small-grid spectra, into G'
    CHK(fast_class_alone(p, COL_ADJ));
    return fast_plane_adj_out(p, rho);
  }
  CHK(launch_small_fwd(p, d));
  CHK(launch_class_adj(p, 0));
  CHK(launch_plane_adj(p, OUT_SCALE_B, rho, nullptr));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_backproject(mh3d_plan_t p, const float* d, float* c) {
  CHK(check_plan(p));
  if (!c || !d) return fail(MH3D_ERR_INVALID, "NULL array");
  CHK(launch_small_fwd_adj(p, d));
  if (use_fast(p)) {
    // column and plane passes of A^T with one descriptor per harmonic (all K at once when
    // their Q buffers fit, else one harmonic after another through the shared one)
    if (p->each_batched) {
      p->fast->adjoint_each(p->ls, p->vdk, p->g.K, c);
      return last_launch("k_fast_col / k_fast_plane_adj (per harmonic)");
    }
    for (int k = 0; k < p->g.K; ++k) {
      p->fast->adjoint_each(p->ls, p->vdk + k, 1, c + (size_t)k * p->g.N);
      CHK(last_launch("k_fast_col / k_fast_plane_adj (per harmonic)"));
    }
    return MH3D_OK;
  }
  for (int k = 0; k < p->g.K; ++k) {
    CHK(launch_class_adj(p, 0, p->vdk + k));
    CHK(launch_plane_adj(p, OUT_SCALE_B, c + (size_t)k * p->g.N, nullptr, p->vdk + k));
  }
  return MH3D_OK;
}

// out = (A^T A + lambda T^T T)(s w): s from the state (1/||w|| in power iteration).
static mh3d_status apply_normal_scaled(mh3d_plan_t p, const float* w, float* out) {
  if (use_fast(p)) {
    CHK(fast_plane_fwd(p, SRC_SCALED, w));
    CHK(fast_class(p, 1, NRM_PLAIN));
    return fast_adjoint_step(p, UPD_NORMAL, out, w);
  }
  CHK(launch_plane_fwd(p, SRC_SCALED, w));
  if (fused_class(p)) {
    CHK(launch_class_normal(p, 1, NRM_PLAIN));
  } else {
    if (p->g.padded) {
      CHK(launch_class_fwd(p, 1, FWD_G));
      CHK(launch_small_inv(p, EPI_BACK, nullptr));   // crop to the field of view
    } else {
      CHK(launch_class_fwd(p, 1, FWD_ADJ));
    }
    CHK(launch_class_adj(p, 1));
  }
  CHK(launch_adjoint_step(p, UPD_NORMAL, out, w));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_normal(mh3d_plan_t p, const float* x, float* out) {
  CHK(check_plan(p));
  SolverPasses sp(p);
  if (!x || !out) return fail(MH3D_ERR_INVALID, "NULL array");
  DevState z;
  memset(&z, 0, sizeof z);
  z.scale = 1.0;
  z.kmax = 1 << 30;
  CHK(state_set(p, z));
  return apply_normal_scaled(p, x, out);
}

static mh3d_status read_state(mh3d_plan_t p, DevState& h) {
  HIPCHK(hipMemcpyAsync(&h, p->st, sizeof h, hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return MH3D_OK;
}

// Power iteration with start vector x0 of Philox uniforms in vol[0] (v_0 = x0/||x0||).
static mh3d_status power_iteration(mh3d_plan_t p, int iters, uint64_t seed, double* lmax) {
  const Geo& g = p->g;
  DevState z;
  memset(&z, 0, sizeof z);
  z.k = 0;
  z.kmax = 1 << 30;
  CHK(state_set(p, z));
  {
    Timer t(p, KID_AUX);
    hipLaunchKernelGGL(k_philox_uniform, dim3(256), dim3(256), 0, p->stream, (long long)g.N, seed, 0u, p->vol[0],
                       p->partials, p->st);
    CHK(last_launch("k_philox_uniform"));
  }
  int cur = 0;
  for (int t = 0; t < iters; ++t) {
    CHK(apply_normal_scaled(p, p->vol[cur], p->vol[1 - cur]));
    cur = 1 - cur;
  }
  DevState h;
  CHK(read_state(p, h));
  if (h.nonfinite != 0.0 || !std::isfinite(h.lmax)) return fail(MH3D_ERR_NONFINITE, "power iteration produced a non-finite value");
  *lmax = h.lmax;
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_power_iteration(mh3d_plan_t p, int32_t iters, uint64_t seed, double* lmax) {
  CHK(check_plan(p));
  SolverPasses sp(p);
  if (!lmax || iters < 1) return fail(MH3D_ERR_INVALID, "bad power-iteration arguments");
  return power_iteration(p, iters, seed, lmax);
}

// ============================================================================ solver
// One accelerated projected gradient update of the plan's volume; buffers and the
// step come from the device state, so the same launches serve every iteration.
// first: the first update of a solve call (with k_step_and_fwd the forward plane pass of
// every later update ran in the previous update's last launch).
static mh3d_status enqueue_update(mh3d_plan_t p, bool first) {
  Timer t(p, KID_SOLVE_ITER);
  if (use_fast(p)) {
    CHK(fast_plane_fwd(p, SRC_FISTA_Y, nullptr));
    CHK(fast_class(p, 1, NRM_RESID));   // against the data's spectra, held in G'
    return fast_adjoint_step(p, UPD_FISTA, nullptr, nullptr);
  }
  if (first || !step_and_fwd(p)) CHK(launch_plane_fwd(p, SRC_FISTA_Y, nullptr));
  if (fused_class(p)) {
    CHK(launch_class_normal(p, 1, NRM_RESID));   // against the data's spectra, held in G'
  } else {
    if (p->g.padded) {
      CHK(launch_class_fwd(p, 1, FWD_G));
      CHK(launch_small_inv(p, EPI_RESID_BACK, nullptr));   // residual on the field of view
    } else {
      CHK(launch_class_fwd(p, 1, FWD_RESID));   // residual spectrum against the data's, held in G
    }
    CHK(launch_class_adj(p, 1));
  }
  if (step_and_fwd(p)) return launch_step_and_fwd(p);
  CHK(launch_adjoint_step(p, UPD_FISTA, nullptr, nullptr));
  return MH3D_OK;
}

static mh3d_status ensure_hist(mh3d_plan_t p, int n) {
  if (p->hist_cap >= n) return MH3D_OK;
  if (p->hist) (void)hipFree(p->hist);
  p->hist = nullptr;
  p->hist_cap = 0;
  HIPCHK(hipMalloc(&p->hist, sizeof(double) * n));
  p->hist_cap = n;
  return MH3D_OK;
}

// Prepares rho^{k0}, y^{k0}, the descriptor and the state of a solve.
// hist: device array of at least opts->max_iter doubles receiving r_k.
static mh3d_status solve_setup(mh3d_plan_t p, const float* d, const float* rho0, const mh3d_solve_opts* opts,
                               double tau, double* hist) {
  const Geo& g = p->g;
  const int k0 = opts->k0;
  HIPCHK(hipMemcpyAsync(p->vol[k0 & 1], rho0, sizeof(float) * g.N, hipMemcpyDeviceToDevice, p->stream));
  {
    Timer t(p, KID_AUX);
    const float* prev = opts->rho_prev ? opts->rho_prev : rho0;
    k_fista_init<<<dim3(1024), dim3(256), 0, p->ls>>>(g.N, rho0, prev, (float)((k0 - 1.0) / (k0 + 2.0)),
                                                            p->vol[2 + (k0 & 1)]);
    CHK(last_launch("k_fista_init"));
  }
  p->vdh.d = d;
  p->vdh.hist = hist;
  p->vdh.hist_len = opts->max_iter;
  p->vdh.k_first = k0;
  CHK(upload_desc(p));
  // without padding the updates form the residual spectrum F(A y) - F(d): F(d) once,
  // held in G for the whole solve (the fused class pass takes it one x' transform
  // further, into G')
  if (!g.padded) CHK(launch_small_fwd(p, d, p->G));
  if (fused_class(p)) {
    Timer t(p, KID_AUX);
    k_class_data<<<dim3(g.ncls / g.cpw), dim3(p->L.T_class), p->L.lds_class, p->ls>>>(p->vda);
    CHK(last_launch("k_class_data"));
  }
  DevState s0;
  memset(&s0, 0, sizeof s0);
  s0.k = k0;
  s0.tau = tau;
  s0.lam = p->desc.lambda;
  s0.tol = opts->rel_tol;
  s0.kmax = k0 + opts->max_iter - 1;
  s0.last_k = k0 - 1;
  CHK(state_set(p, s0));
  return MH3D_OK;
}

static mh3d_status validate_opts(const mh3d_solve_opts* opts) {
  if (!opts) return fail(MH3D_ERR_INVALID, "opts is NULL");
  if (opts->max_iter < 1) return fail(MH3D_ERR_INVALID, "max_iter must be >= 1");
  if (opts->k0 < 1) return fail(MH3D_ERR_INVALID, "k0 must be >= 1");
  if (!(opts->rel_tol >= 0)) return fail(MH3D_ERR_INVALID, "rel_tol must be >= 0");
  return MH3D_OK;
}

static mh3d_status resolve_tau(mh3d_plan_t p, const mh3d_solve_opts* opts, double* tau, double* lmax) {
  *tau = opts->tau;
  *lmax = 0.0;
  if (!(*tau > 0)) {
    // L depends on the operator only: computed once per plan and (iterations, seed)
    const int it = opts->power_iters > 0 ? opts->power_iters : 50;
    if (p->pi_iters == it && p->pi_seed == opts->power_seed) {
      *lmax = p->pi_lmax;
    } else {
      CHK(power_iteration(p, it, opts->power_seed, lmax));
      if (!(*lmax > 0)) return fail(MH3D_ERR_NONFINITE, "power iteration gave L = %g", *lmax);
      p->pi_iters = it;
      p->pi_seed = opts->power_seed;
      p->pi_lmax = *lmax;
    }
    *tau = 1.0 / (1.05 * *lmax);
  }
  return MH3D_OK;
}

static mh3d_status finish_solve(mh3d_plan_t p, float* rho_inout, const mh3d_solve_opts* opts, const DevState& h,
                                double tau, double lmax, float ms, mh3d_solve_info* info, const double* hist) {
  const int iters = h.last_k - opts->k0 + 1;
  if (iters >= 1)
    HIPCHK(hipMemcpyAsync(rho_inout, p->vol[(h.last_k + 1) & 1], sizeof(float) * p->g.N, hipMemcpyDeviceToDevice,
                          p->stream));
  if (opts->history && opts->history_len > 0 && iters > 0) {
    const int n = std::min(iters, (int)opts->history_len);
    HIPCHK(hipMemcpyAsync(opts->history, hist, sizeof(double) * n, hipMemcpyDeviceToHost, p->stream));
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  mh3d_status status = MH3D_OK;
  if (h.nonfinite != 0.0) status = fail(MH3D_ERR_NONFINITE, "non-finite value in the solver reductions");
  else if (opts->rel_tol > 0 && !(h.rel_step <= opts->rel_tol))
    status = fail(MH3D_ERR_NOT_CONVERGED, "r_k = %g > tol after %d updates", h.rel_step, iters);
  if (info) {
    info->iters = iters;
    info->rel_step = h.rel_step;
    info->tau = tau;
    info->lmax = lmax;
    info->ms_total = ms;
    info->ms_per_iter = iters > 0 ? ms / iters : 0.f;
    info->status = status;
  }
  return status;
}

// The updates of a prepared solve: plain launches, a chunk of updates between reads of
// the state.  (A captured graph of the chunk was measured: 1.5 % less time per update at
// 96x96x64, but its capture and instantiation cost more than a whole solve on first use.)
static mh3d_status run_updates(mh3d_plan_t p, const mh3d_solve_opts* opts, DevState& h) {
  const int chunk = opts->check_every > 0 ? opts->check_every : 16;
  memset(&h, 0, sizeof h);
  int issued = 0;
  while (issued < opts->max_iter) {
    const int n = std::min(chunk, opts->max_iter - issued);
    for (int i = 0; i < n; ++i) CHK(enqueue_update(p, issued + i == 0));
    issued += n;
    CHK(read_state(p, h));
    if (h.done) break;
  }
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_solve(mh3d_plan_t p, const float* d, float* rho_inout, const mh3d_solve_opts* opts,
                                  mh3d_solve_info* info) {
  CHK(check_plan(p));
  if (!d || !rho_inout) return fail(MH3D_ERR_INVALID, "NULL argument");
  CHK(validate_opts(opts));
  SolverPasses sp(p);
  EventPair ev;
  HIPCHK(ev.create());
  HIPCHK(hipEventRecord(ev.e0, p->stream));
  double tau, lmax;
  CHK(resolve_tau(p, opts, &tau, &lmax));
  CHK(ensure_hist(p, opts->max_iter));
  CHK(solve_setup(p, d, rho_inout, opts, tau, p->hist));
  DevState h;
  CHK(run_updates(p, opts, h));
  HIPCHK(hipEventRecord(ev.e1, p->stream));
  HIPCHK(hipEventSynchronize(ev.e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ev.e0, ev.e1);
  return finish_solve(p, rho_inout, opts, h, tau, lmax, ms, info, p->hist);
}

// ---------------------------------------------------------------------------- solve without allocation
// The r_k history of mh3d_solve_static: a file-scope device array (each GPU the library
// runs on holds its own copy until the process ends).  Host code never passes the
// array's name to a kernel or a copy: it resolves the device address once per device
// (hipGetSymbolAddress, with that device current) and uses that.
constexpr int kStaticHistory = 1 << 16;   // updates per call (512 KiB per GPU)
static __device__ __align__(256) double scratch[kStaticHistory];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_dev;   // resolved address per device ordinal

static mh3d_status static_history(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_solve_static(mh3d_plan_t p, const float* d, float* rho_inout, const mh3d_solve_opts* opts,
                                         mh3d_solve_info* info) {
  CHK(check_plan(p));
  if (!d || !rho_inout) return fail(MH3D_ERR_INVALID, "NULL argument");
  CHK(validate_opts(opts));
  if (opts->max_iter > kStaticHistory)
    return fail(MH3D_ERR_INVALID, "max_iter = %d exceeds the %d updates of the static history", opts->max_iter,
                kStaticHistory);
  if (p->prof_on) return fail(MH3D_ERR_INVALID, "pass profiling creates events: disable mh3d_profile first");
  double* hist = nullptr;
  CHK(static_history(&hist));
  SolverPasses sp(p);
  const auto t0 = std::chrono::steady_clock::now();
  double tau, lmax;
  CHK(resolve_tau(p, opts, &tau, &lmax));
  CHK(solve_setup(p, d, rho_inout, opts, tau, hist));
  DevState h;
  CHK(run_updates(p, opts, h));
  HIPCHK(hipStreamSynchronize(p->stream));
  const float ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return finish_solve(p, rho_inout, opts, h, tau, lmax, ms, info, hist);
}

// ============================================================================ batch
struct mh3d_batch_s {
  std::vector<mh3d_plan_t> plans;
  hipStream_t stream;
  VolDesc* vds = nullptr;            // device descriptors of all volumes
  std::vector<VolDesc> hvd;          // their host copies (plane passes at one workgroup per plane)
  // plane, class (padded volumes), small (padded volumes), fused class (the others), per-volume
  int2* tasks[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int ntask[5] = {0, 0, 0, 0, 0};
  int T_class = 0, T_small = 0;
  size_t lds_plane = 0, lds_class = 0, lds_small = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap_stream = nullptr;
  int chunk = 0;
};

extern "C" void mh3d_batch_destroy(mh3d_batch_t b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (auto* p : b->plans) p->batch_refs--;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->vds) (void)hipFree(b->vds);
  for (int i = 0; i < 5; ++i)
    if (b->tasks[i]) (void)hipFree(b->tasks[i]);
  delete b;
}

// Appends the n class blocks of volume v so that the tasks one XCD runs (blocks are
// dealt round-robin over the 8 XCDs by launch index) take consecutive classes, whose
// short runs of G, G' and the class-layout spectra share L2 lines.
static void push_xcd_grouped(std::vector<int2>& t, int v, int n) {
  const size_t s = t.size();
  t.resize(s + n);
  int u = 0;
  for (size_t x = 0; x < 8; ++x)
    for (size_t i = s; i < s + (size_t)n; ++i)
      if ((i & 7) == x) t[i] = make_int2(v, u++);
}

extern "C" mh3d_status mh3d_batch_create(int32_t n, const mh3d_plan_t* plans, mh3d_batch_t* out) {
  if (!out) return fail(MH3D_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || !plans) return fail(MH3D_ERR_INVALID, "empty batch");
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(MH3D_ERR_INVALID, "plan %d is NULL", i);
    if (!plans[i]->compact) return fail(MH3D_ERR_UNSUPPORTED, "batched solves need analytic-PSF plans (plan %d)", i);
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(MH3D_ERR_INVALID, "plan %d appears twice in the batch", i);
    // every volume's per-solve setup is enqueued on its own plan's stream and the batch's
    // passes on plans[0]'s: one stream orders them
    if (plans[i]->stream != plans[0]->stream)
      return fail(MH3D_ERR_INVALID, "plan %d uses another stream than plan 0 (a batch runs on one stream)", i);
  }
  mh3d_batch_t b = new mh3d_batch_s();
  b->plans.assign(plans, plans + n);
  for (auto* p : b->plans) p->batch_refs++;
  b->stream = plans[0]->stream;
  std::vector<int2> t[5];
  for (int v = 0; v < n; ++v) {
    const mh3d_plan_t p = plans[v];
    // one workgroup per x-plane: the batch already fills the chip with the planes of
    // many volumes, so splitting planes would only add work
    for (int i = 0; i < p->g.nx; ++i) t[0].push_back(make_int2(v, i));
    // volumes without padding run their class passes as one; the small-grid pass of the
    // updates is needed only to crop to a field of view
    push_xcd_grouped(t[p->g.padded ? 1 : 3], v, p->g.ncls / p->g.cpw);
    if (p->g.padded)
      for (int i = 0; i < p->g.K * (p->g.mx / p->g.xb); ++i) t[2].push_back(make_int2(v, i));
    t[4].push_back(make_int2(v, 0));
    b->T_class = std::max(b->T_class, p->L.T_class);
    b->lds_plane = std::max(b->lds_plane, p->L.lds_plane);
    b->lds_class = std::max(b->lds_class, p->L.lds_class);
    b->lds_small = std::max(b->lds_small, p->L.lds_small);
    if (p->g.padded) b->T_small = std::max(b->T_small, p->L.T_small);
  }
  auto bail = [&](mh3d_status s) { mh3d_batch_destroy(b); return s; };
  if (hipMalloc(&b->vds, sizeof(VolDesc) * n) != hipSuccess) return bail(fail(MH3D_ERR_OOM, "batch descriptors"));
  b->hvd.resize(n);
  for (int i = 0; i < 5; ++i) {
    b->ntask[i] = (int)t[i].size();
    if (t[i].empty()) continue;   // e.g. no padded volume
    if (hipMalloc(&b->tasks[i], sizeof(int2) * t[i].size()) != hipSuccess) return bail(fail(MH3D_ERR_OOM, "batch tasks"));
    if (hipMemcpy(b->tasks[i], t[i].data(), sizeof(int2) * t[i].size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(MH3D_ERR_HIP, "upload of batch tasks failed"));
  }
  *out = b;
  return MH3D_OK;
}

// Device descriptor of volume v: the plan's, with one workgroup per x-plane.
static mh3d_status batch_upload(mh3d_batch_t b, int v) {
  b->hvd[v] = b->plans[v]->vdh;
  b->hvd[v].g.ps = 1;
  b->hvd[v].nb_upd = b->plans[v]->g.nx;   // the step's sums: one plane-pass block per x-plane
  HIPCHK(hipMemcpyAsync(b->vds + v, &b->hvd[v], sizeof(VolDesc), hipMemcpyHostToDevice, b->stream));
  return MH3D_OK;
}

// The class passes of every volume: one fused launch for the volumes without padding,
// then forward class pass, crop (small-grid pass) and adjoint class pass for the padded
// ones.  mode: NRM_RESID (updates) or NRM_PLAIN (power iteration).
static mh3d_status batch_class(mh3d_batch_t b, hipStream_t st, int mode) {
  if (b->ntask[3]) {
    k_class_normal_batch<<<dim3(b->ntask[3]), dim3(b->T_class), b->lds_class, st>>>(b->vds, b->tasks[3], mode);
    CHK(last_launch("k_class_normal_batch"));
  }
  if (b->ntask[1]) {
    k_class_fwd_batch<<<dim3(b->ntask[1]), dim3(b->T_class), b->lds_class, st>>>(b->vds, b->tasks[1], FWD_G);
    CHK(last_launch("k_class_fwd_batch"));
    if (mode == NRM_RESID)
      k_small_inv<EPI_RESID_BACK><<<dim3(b->ntask[2]), dim3(b->T_small), b->lds_small, st>>>(b->vds, b->tasks[2], nullptr);
    else
      k_small_inv<EPI_BACK><<<dim3(b->ntask[2]), dim3(b->T_small), b->lds_small, st>>>(b->vds, b->tasks[2], nullptr);
    CHK(last_launch("k_small_inv (batch)"));
    k_class_adj_batch<<<dim3(b->ntask[1]), dim3(b->T_class), b->lds_class, st>>>(b->vds, b->tasks[1]);
    CHK(last_launch("k_class_adj_batch"));
  }
  return MH3D_OK;
}

// One update of every volume of the batch: three launches over the task tables (three
// more when some volume is padded: its forward class, small-grid and adjoint class
// passes).  The batch runs one workgroup per x-plane, so the step's
// launch also runs the next update's forward plane pass (k_step_and_fwd); the first
// update of a solve call is preceded by batch_first_plane_pass.
static mh3d_status batch_update(mh3d_batch_t b, hipStream_t st) {
  CHK(batch_class(b, st, NRM_RESID));
  AdjOut ao;
  ao.out = nullptr;
  ao.yin = nullptr;
  k_step_and_fwd<<<dim3(b->ntask[0]), dim3(1024), b->lds_plane, st>>>(b->vds, b->tasks[0], ao);
  CHK(last_launch("k_step_and_fwd (batch)"));
  k_vol_finish<UPD_FISTA><<<dim3(b->ntask[4]), dim3(256), 0, st>>>(b->vds, b->tasks[4]);
  CHK(last_launch("k_vol_finish (batch)"));
  return MH3D_OK;
}

static mh3d_status batch_first_plane_pass(mh3d_batch_t b, hipStream_t st) {
  k_plane_fwd<SRC_FISTA_Y><<<dim3(b->ntask[0]), dim3(1024), b->lds_plane, st>>>(b->vds, b->tasks[0], nullptr);
  return last_launch("k_plane_fwd (batch)");
}

// One power-iteration step of every volume: w_{t+1} = N (s w_t), w_t in rho[k & 1].
static mh3d_status batch_power_step(mh3d_batch_t b, hipStream_t st) {
  k_plane_fwd<SRC_SCALED><<<dim3(b->ntask[0]), dim3(1024), b->lds_plane, st>>>(b->vds, b->tasks[0], nullptr);
  CHK(last_launch("k_plane_fwd (batch power)"));
  CHK(batch_class(b, st, NRM_PLAIN));
  AdjOut ao;
  ao.out = nullptr;
  ao.yin = nullptr;
  k_plane_adj<OUT_STEP_NORMAL><<<dim3(b->ntask[0]), dim3(1024), b->lds_plane, st>>>(b->vds, b->tasks[0], ao);
  CHK(last_launch("k_plane_adj (batch power)"));
  k_vol_finish<UPD_NORMAL><<<dim3(b->ntask[4]), dim3(256), 0, st>>>(b->vds, b->tasks[4]);
  CHK(last_launch("k_vol_finish (batch power)"));
  return MH3D_OK;
}

// Step sizes of every volume from batched power iterations (same start vectors and
// recurrence as mh3d_power_iteration on each plan).
static mh3d_status batch_power(mh3d_batch_t b, int iters, uint64_t seed, std::vector<double>& lmax) {
  const int n = (int)b->plans.size();
  for (int v = 0; v < n; ++v) {
    mh3d_plan_t p = b->plans[v];
    DevState z;
    memset(&z, 0, sizeof z);
    z.k = 0;
    z.kmax = iters - 1;
    CHK(state_set(p, z));
    hipLaunchKernelGGL(k_philox_uniform, dim3(256), dim3(256), 0, p->stream, (long long)p->g.N, seed, 0u, p->vol[0],
                       p->partials, p->st);
    CHK(last_launch("k_philox_uniform"));
    CHK(batch_upload(b, v));
  }
  for (int t = 0; t < iters; ++t) CHK(batch_power_step(b, b->stream));
  std::vector<DevState> hs(n);
  for (int v = 0; v < n; ++v)
    HIPCHK(hipMemcpyAsync(&hs[v], b->plans[v]->st, sizeof(DevState), hipMemcpyDeviceToHost, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  lmax.assign(n, 0.0);
  for (int v = 0; v < n; ++v) {
    if (hs[v].nonfinite != 0.0 || !(hs[v].lmax > 0) || !std::isfinite(hs[v].lmax))
      return fail(MH3D_ERR_NONFINITE, "power iteration of volume %d gave L = %g", v, hs[v].lmax);
    lmax[v] = hs[v].lmax;
  }
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_solve_batch(mh3d_batch_t b, const float* const* d, float* const* rho_inout,
                                        const mh3d_solve_opts* opts, mh3d_solve_info* infos) {
  if (!b) return fail(MH3D_ERR_INVALID, "batch is NULL");
  if (!d || !rho_inout) return fail(MH3D_ERR_INVALID, "NULL argument");
  CHK(validate_opts(opts));
  const int n = (int)b->plans.size();
  for (int v = 0; v < n; ++v)
    if (!d[v] || !rho_inout[v]) return fail(MH3D_ERR_INVALID, "NULL array for volume %d", v);
  EventPair ev;
  HIPCHK(ev.create());
  HIPCHK(hipEventRecord(ev.e0, b->stream));
  std::vector<double> tau(n, opts->tau), lmax(n, 0.0);
  if (!(opts->tau > 0)) {
    const int it = opts->power_iters > 0 ? opts->power_iters : 50;
    bool cached = true;
    for (int v = 0; v < n; ++v) {
      const mh3d_plan_t p = b->plans[v];
      if (p->pi_iters == it && p->pi_seed == opts->power_seed) lmax[v] = p->pi_lmax;
      else cached = false;
    }
    if (!cached) {
      CHK(batch_power(b, it, opts->power_seed, lmax));
      for (int v = 0; v < n; ++v) {
        b->plans[v]->pi_iters = it;
        b->plans[v]->pi_seed = opts->power_seed;
        b->plans[v]->pi_lmax = lmax[v];
      }
    }
    for (int v = 0; v < n; ++v) tau[v] = 1.0 / (1.05 * lmax[v]);
  }
  for (int v = 0; v < n; ++v) {
    mh3d_plan_t p = b->plans[v];
    CHK(ensure_hist(p, opts->max_iter));
    CHK(solve_setup(p, d[v], rho_inout[v], opts, tau[v], p->hist));
    CHK(batch_upload(b, v));
  }
  const int chunk = opts->check_every > 0 ? opts->check_every : 16;
  if (!b->gexec || b->chunk != chunk) {
    if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    mh3d_status s = MH3D_OK;
    for (int i = 0; i < chunk && s == MH3D_OK; ++i) s = batch_update(b, b->cap_stream);
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &gr);
    if (s != MH3D_OK) { if (gr) (void)hipGraphDestroy(gr); return s; }
    if (e != hipSuccess) return fail(MH3D_ERR_HIP, "stream capture failed: %s", hipGetErrorString(e));
    b->graph = gr;
    HIPCHK(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->chunk = chunk;
  }
  // per-volume state snapshots after each replay; the graph is replayed until every
  // volume reports done (each volume stops updating at its own r_k <= tol)
  std::vector<DevState> hs(n);
  CHK(batch_first_plane_pass(b, b->stream));
  int issued = 0;
  while (issued < opts->max_iter) {
    HIPCHK(hipGraphLaunch(b->gexec, b->stream));
    issued += chunk;
    bool all = true;
    for (int v = 0; v < n; ++v)
      HIPCHK(hipMemcpyAsync(&hs[v], b->plans[v]->st, sizeof(DevState), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int v = 0; v < n; ++v) all = all && hs[v].done;
    if (all) break;
  }
  HIPCHK(hipEventRecord(ev.e1, b->stream));
  HIPCHK(hipEventSynchronize(ev.e1));
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, ev.e0, ev.e1);
  mh3d_status worst = MH3D_OK;
  for (int v = 0; v < n; ++v) {
    mh3d_solve_info inf;
    mh3d_solve_opts o = *opts;
    o.history = nullptr;
    o.history_len = 0;
    mh3d_status s = finish_solve(b->plans[v], rho_inout[v], &o, hs[v], tau[v], lmax[v], ms, &inf, b->plans[v]->hist);
    if (infos) infos[v] = inf;
    if (s != MH3D_OK && worst == MH3D_OK) worst = s;
  }
  return worst;
}

// ============================================================================ export / profile
extern "C" mh3d_status mh3d_plan_export(mh3d_plan_t p, mh3d_field field, void* dst, size_t* bytes) {
  CHK(check_plan(p));
  const Geo& g = p->g;
  size_t need = 0;
  switch (field) {
    case MH3D_FIELD_PROFILE: need = sizeof(double) * g.K * g.nx; break;
    case MH3D_FIELD_ENVELOPE: need = sizeof(double) * (size_t)g.ny * g.nz; break;
    case MH3D_FIELD_SENS: need = sizeof(float) * g.C * g.N; break;
    case MH3D_FIELD_SPECTRUM: need = sizeof(float2) * (size_t)g.C * g.K * g.nx * g.ny * g.nzh; break;
    default: return fail(MH3D_ERR_INVALID, "unknown field %d", (int)field);
  }
  if (bytes) *bytes = need;
  if (!dst) return MH3D_OK;
  if ((field == MH3D_FIELD_PROFILE || field == MH3D_FIELD_ENVELOPE) && !p->compact)
    return fail(MH3D_ERR_INVALID, "plan uses a user PSF; no analytic profile/envelope");
  switch (field) {
    case MH3D_FIELD_PROFILE: HIPCHK(hipMemcpyAsync(dst, p->prof, need, hipMemcpyDeviceToDevice, p->stream)); break;
    case MH3D_FIELD_ENVELOPE: HIPCHK(hipMemcpyAsync(dst, p->env, need, hipMemcpyDeviceToDevice, p->stream)); break;
    case MH3D_FIELD_SENS: HIPCHK(hipMemcpyAsync(dst, p->b, need, hipMemcpyDeviceToDevice, p->stream)); break;
    default:
      for (int c = 0; c < g.C; ++c) {
        const size_t esz = p->compact ? sizeof(float) : sizeof(float2);
        hipLaunchKernelGGL(k_spectrum_export, dim3(1024), dim3(256), 0, p->stream, g,
                           (const char*)p->hs + (size_t)c * g.K * g.hsz * esz, p->imag_mask, p->compact,
                           reinterpret_cast<float2*>(dst) + (size_t)c * g.K * g.nx * g.ny * g.nzh);
        CHK(last_launch("k_spectrum_export"));
      }
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  if (!ctr || !key || !out) return fail(MH3D_ERR_INVALID, "NULL argument");
  uint32_t* d = nullptr;
  HIPCHK(hipMalloc(&d, 4 * sizeof(uint32_t)));
  hipLaunchKernelGGL(k_philox_words, dim3(1), dim3(64), 0, 0, ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], d);
  mh3d_status s = last_launch("k_philox_words");
  if (s == MH3D_OK && hipMemcpy(out, d, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
    s = fail(MH3D_ERR_HIP, "copy of Philox words failed");
  (void)hipFree(d);
  return s;
}

extern "C" mh3d_status mh3d_profile(mh3d_plan_t p, int32_t enable) {
  CHK(check_plan(p));
  drain_events(p);
  p->prof_on = enable != 0;
  memset(p->ms, 0, sizeof p->ms);
  memset(p->launches, 0, sizeof p->launches);
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_profile_read(mh3d_plan_t p, mh3d_profile_data* out) {
  CHK(check_plan(p));
  if (!out) return fail(MH3D_ERR_INVALID, "out is NULL");
  HIPCHK(hipStreamSynchronize(p->stream));
  drain_events(p);
  for (int i = 0; i < MH3D_NKERNEL; ++i) {
    out->ms[i] = p->ms[i];
    out->launches[i] = p->launches[i];
    out->name[i] = kKernelNames[i];
  }
  return MH3D_OK;
}

// ============================================================================ warm-start network
// ============================================================================ MHAD
extern "C" mh3d_status mh3d_mhad(mh3d_plan_t p, const float* d, double lambda, const double* c, float* out) {
  CHK(check_plan(p));
  if (!d || !out) return fail(MH3D_ERR_INVALID, "NULL array");
  if (!(lambda > 0.0) || !(lambda < 1e300)) return fail(MH3D_ERR_INVALID, "MHAD needs a finite lambda > 0");
  const Geo& g = p->g;
  const int m = g.mxf;
  if (!is_23_smooth(m)) return fail(MH3D_ERR_UNSUPPORTED, "MHAD needs a drive-axis portrait length 2^a 3^b (got %d)", m);
  MhadW wk;
  memset(&wk, 0, sizeof wk);
  for (int i = 0; i < g.K; ++i) {
    wk.ord[i] = p->harm[i] + p->desc.order_offset - 1;
    const double ck = c ? c[i] : 1.0;
    if (!(ck != 0.0) || !std::isfinite(ck)) return fail(MH3D_ERR_INVALID, "c[%d] must be finite and nonzero", i);
    wk.cinv[i] = 1.0 / ck;
  }
  const int ls = pad_odd(m);
  const int CB = std::max(1, std::min(32, (int)(60 * 1024 / (24 * (size_t)ls))));
  const long long C = (long long)g.myf * g.mzf;
  const size_t lds = sizeof(float2) * ((size_t)m + 3 * (size_t)CB * ls) + sizeof(float) * m;
  k_mhad<<<dim3((unsigned)((C + CB - 1) / CB)), dim3(256), lds, p->stream>>>(d, g.K, wk, lambda, m, C, CB, out);
  return last_launch("k_mhad");
}

// ============================================================================ pass timing
extern "C" mh3d_status mh3d_time_pass(mh3d_plan_t p, int32_t pass, int32_t reps, double* us) {
  CHK(check_plan(p));
  if (pass < 0 || pass > 7 || reps < 1 || !us) return fail(MH3D_ERR_INVALID, "bad pass timing arguments");
  if (pass >= 6 && !fused_class(p))
    return fail(MH3D_ERR_UNSUPPORTED, "the plan runs no fused class pass (vector model or boundary padding)");
  if (p->prof_on) return fail(MH3D_ERR_INVALID, "disable mh3d_profile before timing passes");
  float* dtmp = nullptr;
  HIPCHK(hipMalloc(&dtmp, sizeof(float) * (size_t)p->g.K * p->g.M));
  (void)hipMemsetAsync(p->vol[0], 0, sizeof(float) * p->g.N, p->stream);
  (void)hipMemsetAsync(dtmp, 0, sizeof(float) * (size_t)p->g.K * p->g.M, p->stream);
  const bool fast = use_fast(p);
  auto launch = [&]() -> mh3d_status {
    // the compile-time passes where the plan has them
    if (fast && pass == 0) return fast_plane_fwd(p, SRC_PLAIN, p->vol[0]);
    if (fast && pass == 1) return fast_class_alone(p, COL_FWD);
    if (fast && pass == 2) return fast_small_inv(p, dtmp);
    if (fast && pass == 3) return launch_small_fwd_adj(p, dtmp);
    if (fast && pass == 4) return fast_class_alone(p, COL_ADJ);
    if (fast && pass == 5) return fast_plane_adj_out(p, p->vol[1]);
    if (fast && pass == 6) return fast_class(p, 0, NRM_STORE);
    if (fast && pass == 7) return fast_adj_and_store(p, dtmp, p->vol[1]);
    switch (pass) {
      case 0: return launch_plane_fwd(p, SRC_PLAIN, p->vol[0]);
      case 1: return launch_class_fwd(p, 0, FWD_G);
      case 2: return launch_small_inv(p, EPI_STORE, dtmp);
      case 3: return launch_small_fwd(p, dtmp);
      case 4: return launch_class_adj(p, 0);
      case 6: return launch_class_normal(p, 0, NRM_STORE);
      case 7: return launch_adj_and_store(p, dtmp, p->vol[1]);
      default: return launch_plane_adj(p, OUT_SCALE_B, p->vol[1], nullptr);
    }
  };
  mh3d_status s = MH3D_OK;
  // the passes' inputs: one full A and A^T first so every intermediate buffer is set
  s = mh3d_forward(p, p->vol[0], dtmp);
  if (s == MH3D_OK) s = mh3d_adjoint(p, dtmp, p->vol[1]);
  if (s == MH3D_OK && fast) s = mh3d_forward_adjoint(p, p->vol[0], dtmp, p->vol[1]);
  for (int i = 0; i < 3 && s == MH3D_OK; ++i) s = launch();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (s == MH3D_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    s = fail(MH3D_ERR_HIP, "event creation failed");
  if (s == MH3D_OK) {
    (void)hipEventRecord(e0, p->stream);
    for (int i = 0; i < reps && s == MH3D_OK; ++i) s = launch();
    (void)hipEventRecord(e1, p->stream);
    float ms = 0.f;
    if (s == MH3D_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      s = fail(MH3D_ERR_HIP, "timing events failed");
    *us = 1e3 * (double)ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(dtmp);
  return s;
}

// ============================================================================ tiles and autotuning
static mh3d_status apply_tiles(mh3d_plan_t p, const mh3d_tiles* t) {
  if (p->batch_refs) return fail(MH3D_ERR_INVALID, "the plan belongs to a batch; set its tiles before creating the batch");
  Geo g = p->g;
  Launch L = p->L;
  CHK(derive_tiles(g, L, t ? t->E : 0, t ? t->cpw : 0, t ? t->xb : 0, t ? t->ps : 0));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->g = g;
  p->L = L;
  p->vda = p->vdd;
  p->psa = p->ps_solve = g.ps;   // the solver's split follows; the autotuner may change it
  fill_desc(p);
  CHK(upload_desc(p));
  CHK(upload_harmonic_descs(p));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_plan_set_tiles(mh3d_plan_t p, const mh3d_tiles* tiles) {
  CHK(check_plan(p));
  return apply_tiles(p, tiles);
}

extern "C" mh3d_status mh3d_plan_get_tiles(mh3d_plan_t p, mh3d_tiles* tiles) {
  CHK(check_plan(p));
  if (!tiles) return fail(MH3D_ERR_INVALID, "tiles is NULL");
  tiles->E = p->g.E;
  tiles->cpw = p->g.cpw;
  tiles->xb = p->g.xb;
  tiles->ps = p->g.ps;
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_plan_path(mh3d_plan_t p, int32_t request, int32_t* active) {
  CHK(check_plan(p));
  if (request < -1 || request > 1) return fail(MH3D_ERR_INVALID, "path request must be -1, 0 or 1");
  if (request >= 0 && (request == 1) != p->fast_on) {
    if (p->batch_refs) return fail(MH3D_ERR_INVALID, "the plan belongs to a batch");
    HIPCHK(hipStreamSynchronize(p->stream));
    p->fast_on = request == 1;
    CHK(upload_desc(p));   // the solver's step sums come from the active path's blocks
  }
  if (active) *active = use_fast(p) ? 1 : 0;
  return MH3D_OK;
}

// Cache key: device architecture, grid, harmonic count, decimation, spectrum form, pass family.
static std::string tune_key(mh3d_plan_t p, bool compiled) {
  int dev = 0;
  std::string arch = "unknown";
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch = arch.substr(0, c);
  }
  char buf[160];
  // plans on the compile-time passes time a different A + A^T (only xb matters there):
  // their own entries
  snprintf(buf, sizeof buf, "%s|%dx%dx%d|K%d|ds%dx%dx%d|%s%s", arch.c_str(), p->g.nx, p->g.ny, p->g.nz, p->g.K, p->g.sx,
           p->g.sy, p->g.sz, p->compact ? "analytic" : (p->g.C > 1 ? (p->g.C == 2 ? "user2" : "user3") : "user"),
           compiled ? "|compiled" : "");
  return buf;
}

struct TuneEntry {
  int E, cpw, xb, ps, ps_solve, tm;
  double us;
};

// The cache is a JSON object, one entry per line:
//   "key": {"E": e, "cpw": c, "xb": x, "ps": s, "ps_solve": q, "tm": m, "us": t},
// (entries without ps_solve take ps for it; without tm, the default threads of the
// merged adjoint launch).
// Lines that do not parse are ignored (the file is rewritten on the next store).
static std::map<std::string, TuneEntry> tune_read(const char* path) {
  std::map<std::string, TuneEntry> m;
  FILE* f = fopen(path, "r");
  if (!f) return m;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char key[256];
    TuneEntry e;
    e.tm = 0;
    if (sscanf(line,
               " \"%255[^\"]\": {\"E\": %d, \"cpw\": %d, \"xb\": %d, \"ps\": %d, \"ps_solve\": %d, \"tm\": %d, \"us\": %lf}",
               key, &e.E, &e.cpw, &e.xb, &e.ps, &e.ps_solve, &e.tm, &e.us) == 8) {
      m[key] = e;
    } else if (sscanf(line, " \"%255[^\"]\": {\"E\": %d, \"cpw\": %d, \"xb\": %d, \"ps\": %d, \"ps_solve\": %d, \"us\": %lf}",
                      key, &e.E, &e.cpw, &e.xb, &e.ps, &e.ps_solve, &e.us) == 7) {
      m[key] = e;
    } else if (sscanf(line, " \"%255[^\"]\": {\"E\": %d, \"cpw\": %d, \"xb\": %d, \"ps\": %d, \"us\": %lf}", key,
                      &e.E, &e.cpw, &e.xb, &e.ps, &e.us) == 6) {
      e.ps_solve = e.ps;
      m[key] = e;
    }
  }
  fclose(f);
  return m;
}

static void tune_write(const char* path, const std::map<std::string, TuneEntry>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) {
    fprintf(f, "  \"%s\": {\"E\": %d, \"cpw\": %d, \"xb\": %d, \"ps\": %d, \"ps_solve\": %d, \"tm\": %d, \"us\": %.3f}%s\n",
            kv.first.c_str(), kv.second.E, kv.second.cpw, kv.second.xb, kv.second.ps, kv.second.ps_solve, kv.second.tm,
            kv.second.us, ++i < m.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  (void)rename(tmp.c_str(), path);
}

// Microseconds per A + A^T application (mh3d_forward_adjoint) with the plan's current
// tiles: HIP events, best of two batches of 8 after 2 warm-up applications.
static mh3d_status time_application(mh3d_plan_t p, float* dtmp, double* us) {
  for (int i = 0; i < 2; ++i) CHK(mh3d_forward_adjoint(p, p->vol[0], dtmp, p->vol[1]));
  EventPair ev;
  HIPCHK(ev.create());
  double best = 1e30;
  mh3d_status s = MH3D_OK;
  for (int r = 0; r < 2 && s == MH3D_OK; ++r) {
    (void)hipEventRecord(ev.e0, p->stream);
    for (int i = 0; i < 8 && s == MH3D_OK; ++i) s = mh3d_forward_adjoint(p, p->vol[0], dtmp, p->vol[1]);
    (void)hipEventRecord(ev.e1, p->stream);
    float ms = 0.f;
    if (hipEventSynchronize(ev.e1) != hipSuccess || hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess)
      s = fail(MH3D_ERR_HIP, "timing events failed");
    best = std::min(best, 1e3 * ms / 8.0);
  }
  *us = best;
  return s;
}

// Microseconds per solver update with the plan's current solver split: solves of 48
// updates with a fixed step and no stopping rule on data d from rho = 0 (the solve's
// own stream timing, setup included), the faster of two kept.
static mh3d_status time_updates(mh3d_plan_t p, const float* d, float* rho, double* us) {
  double best = 1e30;
  for (int r = 0; r < 2; ++r) {
    HIPCHK(hipMemsetAsync(rho, 0, sizeof(float) * p->g.N, p->stream));
    mh3d_solve_opts o;
    memset(&o, 0, sizeof o);
    o.max_iter = 48;
    o.tau = 1e-3;
    o.k0 = 1;
    o.check_every = 48;
    mh3d_solve_info info;
    const mh3d_status s = mh3d_solve(p, d, rho, &o, &info);
    if (s != MH3D_OK && s != MH3D_ERR_NOT_CONVERGED) return s;
    best = std::min(best, 1e3 * (double)info.ms_total / o.max_iter);
  }
  *us = best;
  return MH3D_OK;
}

static bool valid_ps(const Geo& g, int ps) { return ps >= 1 && ps <= 4 && ps <= g.nzh && ps <= g.npairs; }

// Applies the cache's entry for key; false if there is none or it no longer fits the
// shape rules (then it is tuned again).
static bool apply_cached(mh3d_plan_t p, const char* cache_path, const std::string& key, mh3d_tiles* tiles,
                         double* us_out) {
  if (!cache_path) return false;
  const auto m = tune_read(cache_path);
  const auto it = m.find(key);
  if (it == m.end()) return false;
  mh3d_tiles t{it->second.E, it->second.cpw, it->second.xb, it->second.ps};
  if (apply_tiles(p, &t) != MH3D_OK) return false;
  if (valid_ps(p->g, it->second.ps_solve)) {
    p->ps_solve = it->second.ps_solve;
    if (upload_desc(p) != MH3D_OK) return false;
  }
  if (it->second.tm == 512 || it->second.tm == 1024) p->L.T_merge = it->second.tm;
  if (tiles) *tiles = t;
  if (us_out) *us_out = it->second.us;
  return true;
}

// Tiles of the general passes: the cache's entry, else timed (class tiles, then the
// small-grid tiles, the plane split and the merged launch's threads, then the solver's
// split) and stored.
static mh3d_status tune_general(mh3d_plan_t p, const char* cache_path, mh3d_tiles* tiles, double* us_out) {
  const std::string key = tune_key(p, false);
  if (apply_cached(p, cache_path, key, tiles, us_out)) return MH3D_OK;
  const Geo g0 = p->g;
  float* dtmp = nullptr;
  float* rtmp = nullptr;
  HIPCHK(hipMalloc(&dtmp, sizeof(float) * (size_t)g0.K * g0.M));
  if (hipMalloc(&rtmp, sizeof(float) * g0.N) != hipSuccess) {
    (void)hipFree(dtmp);
    return fail(MH3D_ERR_OOM, "autotuner volume");
  }
  (void)hipMemsetAsync(p->vol[0], 0, sizeof(float) * g0.N, p->stream);
  auto run = [&]() -> mh3d_status {
    // phase 1: class tiles (E, cpw) with the heuristic xb; per E the smallest cpw
    // reaching 64, 128, 256 and 512 threads
    std::vector<mh3d_tiles> cands;
    for (int e = 1; e <= g0.S; ++e) {
      if (!valid_E(g0.S, e)) continue;
      int last = 0;
      for (int thr : {64, 128, 256, 512}) {
        for (int c = 1; c <= g0.ncls; ++c) {
          if (g0.ncls % c) continue;
          const long T = (long)c * g0.mx * g0.S / e;
          if (T > 1024) break;
          if (T >= thr || (thr == 64 && c == g0.ncls)) {
            if (c != last) cands.push_back(mh3d_tiles{e, c, 0, 0});
            last = c;
            break;
          }
        }
      }
    }
    mh3d_tiles best{0, 0, 0, 0};
    int best_tm = 0;
    double best_us = 1e30;
    // tm: threads of the merged adjoint launch (0: the default for the tiles)
    auto trial = [&](const mh3d_tiles& t, int tm) -> mh3d_status {
      if (apply_tiles(p, &t) != MH3D_OK) return MH3D_OK;       // shape does not fit: skip
      if (tm) p->L.T_merge = tm;
      double us = 0;
      CHK(time_application(p, dtmp, &us));
      if (us < best_us) { best_us = us; best = t; best.xb = p->g.xb; best.ps = p->g.ps; best_tm = p->L.T_merge; }
      return MH3D_OK;
    };
    for (const auto& t : cands) CHK(trial(t, 0));
    // phase 2: small-grid tiles xb, workgroups per x-plane ps and the merged launch's
    // threads together, with the best class tiles (the small-grid blocks can share a
    // launch with the plane blocks, so the best xb depends on ps and on how many blocks
    // fit beside them)
    const mh3d_tiles cls = best;
    for (int xb : {1, 2, 4, 8, 16, 32}) {
      if (g0.mx % xb) continue;
      for (int ps : {1, 2, 4}) {
        if (ps > g0.nzh || ps > g0.npairs) continue;
        for (int tm : {512, 1024}) CHK(trial(mh3d_tiles{cls.E, cls.cpw, xb, ps}, tm));
      }
    }
    if (best_us >= 1e30) return fail(MH3D_ERR_UNSUPPORTED, "no tile shape could be timed");
    CHK(apply_tiles(p, &best));
    p->L.T_merge = best_tm;
    // phase 3: the solver's plane split, timed on solver updates (which run no
    // small-grid pass, and with ps = 1 start the next update in the step's launch, so
    // their best split can differ); data: A applied to the sensitivity map
    CHK(mh3d_forward(p, p->b, dtmp));
    int best_pss = best.ps;
    double best_nus = 1e30;
    for (int ps : {1, 2, 4}) {
      if (!valid_ps(p->g, ps)) continue;
      p->ps_solve = ps;
      CHK(upload_desc(p));
      double us = 0;
      CHK(time_updates(p, dtmp, rtmp, &us));
      if (us < best_nus) { best_nus = us; best_pss = ps; }
    }
    p->ps_solve = best_pss;
    CHK(upload_desc(p));
    // A + A^T runs its forward plane pass with that split: its time as the plan now runs it
    CHK(time_application(p, dtmp, &best_us));
    if (tiles) *tiles = best;
    if (us_out) *us_out = best_us;
    if (cache_path) {
      auto m = tune_read(cache_path);
      m[key] = TuneEntry{best.E, best.cpw, best.xb, best.ps, best_pss, best_tm, best_us};
      tune_write(cache_path, m);
    }
    return MH3D_OK;
  };
  mh3d_status s = run();
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(dtmp);
  (void)hipFree(rtmp);
  if (s != MH3D_OK) {
    mh3d_tiles h{g0.E, g0.cpw, g0.xb, g0.ps};
    (void)apply_tiles(p, &h);
  }
  return s;
}

static mh3d_status set_fast_on(mh3d_plan_t p, bool on) {
  HIPCHK(hipStreamSynchronize(p->stream));
  p->fast_on = on;
  return upload_desc(p);   // the solver's step sums come from the active path's blocks
}

// Plans on the compile-time passes take only xb from the tiles in their operator calls
// and solves, but a batch runs such a plan's volume on the general passes.  So the
// general tiles come first (timed with the compile-time passes switched off, stored under
// the general key), then xb alone on the compile-time A + A^T; the "|compiled" entry is
// the general tiles with that xb (a batch's general small-grid pass runs that xb too).
extern "C" mh3d_status mh3d_autotune(mh3d_plan_t p, const char* cache_path, mh3d_tiles* tiles, double* us_out) {
  CHK(check_plan(p));
  if (p->batch_refs) return fail(MH3D_ERR_INVALID, "the plan belongs to a batch; tune it before creating the batch");
  if (!(p->fast && p->fast_on)) return tune_general(p, cache_path, tiles, us_out);
  const std::string key = tune_key(p, true);
  if (apply_cached(p, cache_path, key, tiles, us_out)) return MH3D_OK;
  CHK(set_fast_on(p, false));
  mh3d_status s = tune_general(p, cache_path, nullptr, nullptr);
  const mh3d_status s_on = set_fast_on(p, true);
  CHK(s);
  CHK(s_on);
  const mh3d_tiles gen{p->g.E, p->g.cpw, p->g.xb, p->g.ps};
  const int pss = p->ps_solve, tm = p->L.T_merge;
  auto with_xb = [&](int xb) -> mh3d_status {
    mh3d_tiles t = gen;
    t.xb = xb;
    CHK(apply_tiles(p, &t));
    p->ps_solve = pss;
    p->L.T_merge = tm;
    return upload_desc(p);
  };
  float* dtmp = nullptr;
  HIPCHK(hipMalloc(&dtmp, sizeof(float) * (size_t)p->g.K * p->g.M));
  (void)hipMemsetAsync(p->vol[0], 0, sizeof(float) * p->g.N, p->stream);
  int best_xb = 0;
  double best_us = 1e30;
  for (int xb : {1, 2, 4, 8}) {
    if (p->g.mx % xb || with_xb(xb) != MH3D_OK || !use_fast(p)) continue;
    double us = 0;
    s = time_application(p, dtmp, &us);
    if (s != MH3D_OK) break;
    if (us < best_us) { best_us = us; best_xb = xb; }
  }
  if (s == MH3D_OK && best_xb == 0) s = fail(MH3D_ERR_UNSUPPORTED, "no x'-block could be timed on the compile-time passes");
  if (s == MH3D_OK) s = with_xb(best_xb);
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(dtmp);
  if (s != MH3D_OK) {
    (void)with_xb(gen.xb);
    return s;
  }
  if (tiles) *tiles = mh3d_tiles{gen.E, gen.cpw, best_xb, gen.ps};
  if (us_out) *us_out = best_us;
  if (cache_path) {
    auto m = tune_read(cache_path);
    m[key] = TuneEntry{gen.E, gen.cpw, best_xb, gen.ps, pss, tm, best_us};
    tune_write(cache_path, m);
  }
  return MH3D_OK;
}

#include "net_host.hpp"
