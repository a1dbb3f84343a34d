// HIP kernels of the MH3D operator A = P H B, its adjoint and the solver updates.
//
// Pipeline of one application of A (Sec. 4.1 eq. dN, Table tab:ops):
//   plane_fwd  one workgroup per x-plane: u = b . rho, 2-D R2C FFT over (y, z) in
//              LDS, written in the alias-class layout (see geo.hpp)            [B, F_yz]
//   class_fwd  one workgroup per group of classes: FFT along x, multiply by every
//              precomputed spectrum H_k, fold the aliases (P in Fourier form),
//              inverse FFT along the decimated x                                [F_x, H, P]
//   small_inv  one workgroup per (k, block of x'): 2-D C2R over (y', z') of the
//              decimated spectrum -> portrait d_k (optionally minus data)         [F^-1]
// The adjoint runs the same passes backwards (small_fwd, class_adj, plane_adj):
// F(P^T r) tiles the small spectrum, H_k^T multiplies by conj(H_k), and the sum
// over k happens in registers before the inverse x FFT.
//
// Spectra are scaled by 1/N at plan time, so every FFT here is unnormalised.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"
#include "geo.hpp"
#include "langevin_dev.hpp"

namespace mh3d {

// ============================================================================ helpers
// Class-layout index of the full-grid half-plane position (qy, qz), qz <= nz/2,
// and whether the stored value is the conjugate.
__device__ __forceinline__ int class_index_of(const Geo& g, int qy, int qz, bool& cj) {
  const int qzr = (int)g.f_mz.mod((uint32_t)qz);
  int yy = qy, zz = qz;
  cj = false;
  if (2 * qzr > g.mz) {            // stored as the conjugate of (ny - qy, nz - qz)
    yy = qy == 0 ? 0 : g.ny - qy;
    zz = g.nz - qz;
    cj = true;
  }
  const int yq = (int)g.f_my.div((uint32_t)yy), zq = (int)g.f_mz.div((uint32_t)zz);
  const int c = (yy - yq * g.my) * g.mzh + (zz - zq * g.mz);
  const int m = yq * g.sz + zq;
  return c * g.nmem + m;
}

// Source position (qy, qz <= nz/2) in a half plane of the class-layout element e,
// and whether the element is the conjugate of that position.
__device__ __forceinline__ int halfplane_of_member(const Geo& g, int e, bool& cj) {
  const int c = e / g.nmem, m = e % g.nmem;
  const int qy = (c / g.mzh) + (m / g.sz) * g.my;
  const int qz = (c % g.mzh) + (m % g.sz) * g.mz;
  if (2 * qz <= g.nz) { cj = false; return qy * g.nzh + qz; }
  cj = true;
  return ((g.ny - qy) % g.ny) * g.nzh + (g.nz - qz);
}

// LDS line strides: transforms run on contiguous lines padded to an odd length so
// that the transposing passes between them hit distinct banks.
__host__ __device__ inline int pad_odd(int n) { return (n & 1) ? n : n + 1; }

// Complex elements of one LDS buffer of the x-plane kernels: packed row pairs
// [npairs][lsz], half-spectrum columns [nzh][lsy], or a staged class-layout plane.
__host__ __device__ inline int plane_lds(const Geo& g) {
  const int a = g.npairs * pad_odd(g.nz), b = g.nzh * g.lsy, c = g.plane;
  const int m = a > b ? a : b;
  return m > c ? m : c;
}
// One LDS buffer of the small-grid kernels: row pairs [spairs][lsmz] or
// columns [xb*mzh][lsmy].
__host__ __device__ inline int small_lds(const Geo& g) {
  const int a = g.spairs * pad_odd(g.mz), b = g.xb * g.mzh * g.lsmy;
  return a > b ? a : b;
}

// Deterministic block reduction of NV doubles; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_reduce_f64(double* v, double* sh) {
  // sh: >= NV * (blockDim.x / 64 + 1) doubles
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double x = v[j];
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    v[j] = x;
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) sh[j * nw + wid] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[j * nw + w];
      v[j] = s;
    }
  }
  __syncthreads();
}

// Strided block loop with U independent loads in flight per thread: all loads of a
// batch are issued before any result is used (a plain strided loop would wait for
// each load in turn).
template <int U, typename T, typename LD, typename ST>
__device__ __forceinline__ void batched(int n, LD ld, ST st) {
  const int nt = blockDim.x;
  for (int p0 = threadIdx.x; p0 < n; p0 += U * nt) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * nt;
      if (p < n) v[u] = ld(p);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * nt;
      if (p < n) st(p, v[u]);
    }
  }
}

// x-plane (or other unit) handled by block b of nx: consecutive units go to the same
// XCD (blocks are dealt round-robin over the 8 XCDs), so neighbours share an L2.
__device__ __forceinline__ int plane_of_block(int b, int nx) {
  if (nx % 8) return b;
  return (b & 7) * (nx >> 3) + (b >> 3);
}

// Solver / power-iteration state kept in device memory so that a captured
// sequence of launches can be replayed.
struct DevState {
  int k;            // FISTA iteration index of the current y^k
  int done;         // 1 once r_k <= tol or the iteration cap was reached
  int last_k;       // iteration of the last performed update
  int counter;      // arrivals for the last-block reduction
  double tau, lam, tol;
  int kmax;         // last iteration index allowed (k0 + max_iter - 1)
  int pad;
  double rel_step;  // last r_k
  double scale;     // power iteration: 1/||w_{t-1}||
  double lmax;      // power iteration: latest Rayleigh quotient
  double nonfinite;
};

// Everything a pass needs about one volume, in device memory.  The solver's
// iterates rotate by the parity of the device-side iteration counter st->k, so a
// recorded sequence of launches stays valid on replay.
struct VolDesc {
  Geo g;
  const void* hs;          // spectra in the class layout (scaled by 1/N)
  uint32_t imag_mask;      // compact spectra: bit k set -> harmonic k is imaginary
  int compact;
  const float* b;          // sensitivity
  float2* uperm;           // class-layout yz spectra (forward) / adjoint spectra
  float2* G;               // decimated spectra (forward)
  float2* Gp;              // decimated spectra (adjoint)
  float* rho[2];           // FISTA iterates rho^k in rho[k & 1]
  float* y[2];             // FISTA extrapolated points y^k in y[k & 1]
  const float* d;          // FISTA data
  const float2* tw;        // FP32 twiddle tables, offsets off[] for nx, ny, nz, mx, my, mz
  int off[6];
  DevState* st;
  double* partials;        // per-block FP64 partial sums of the x-plane passes
  double* hist;            // FISTA r_k history, index k - k_first
  int hist_len, k_first;
  int reg_kind;
  float lam;
  int T_class;             // threads of the class passes doing element work
  float* u;                // A^T A part of the current step (k_plane_adj<OUT_U> -> k_vol_update)
  float alpha;             // boundary prior weight (eq. finalR), 0 = off
  int aw;                  // its shell depth in voxels
  int nb_upd;              // blocks of k_vol_update for this volume
  // Vector model (components i of the PSF vector and of the sensitivity): component
  // i's spectra at hs + i * hs_cstride elements, its sensitivity at b + i * N and its
  // class-layout spectra at uperm + i * hsz.  ncomp = 1 is the scalar model.
  int ncomp;
  long long hs_cstride;
  // bit k of cmask[i]: component i of harmonic k is present (a PSF block that is
  // identically zero is skipped: no spectrum load, no product)
  uint32_t cmask[3];
  // Separable analytic spectra (the compile-time passes of fast.hpp): the x factors
  // sfs[k][qx], the y-residue table set[y0][q'y][qz], and their intermediates, both in
  // uperm's memory: cp[y0][column][x] (the plane pass's folded shares) and
  // qx[column][x] (the column pass's output for the adjoint plane pass).
  const float* sfs;
  const float2* set;
  float2* cp;
  float2* qx;
};

// Volume and local block index of this block: task table (batched launches) or
// the single volume vds[0].
__device__ __forceinline__ const VolDesc& vol_of(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                 int& lb) {
  if (tasks) {
    const int2 t = tasks[blockIdx.x];
    lb = t.y;
    return vds[t.x];
  }
  lb = blockIdx.x;
  return vds[0];
}

// ============================================================================ pass 1: x-plane R2C
enum { SRC_PLAIN = 0, SRC_RAW = 1, SRC_FISTA_Y = 2, SRC_SCALED = 3 };

// Value fed to the forward FFT at flat voxel i.
template <int SRC>
__device__ __forceinline__ float plane_source(long long i, const float* __restrict__ a,
                                              const float* __restrict__ a2,
                                              const float* __restrict__ b, float coef) {
  if constexpr (SRC == SRC_PLAIN) return b[i] * a[i];
  else if constexpr (SRC == SRC_RAW) return a[i];
  else if constexpr (SRC == SRC_FISTA_Y) return b[i] * a[i];   // a = y^k, skipped once done
  else return b[i] * (coef * a[i]);                             // SRC_SCALED
}

// Row <-> column addressing of the R2C/C2R helpers.  Row r of the real data maps
// to the half-spectrum column layout X[col(r, q)]: col(r, q) = colbase(r) + q * qstride.
struct RowCols {
  int qstride;        // stride between consecutive q of one row
  int per_blk;        // rows per block (my for the small kernels, nrows otherwise)
  FastDiv f_blk;      // divides by per_blk
  int blk_stride;     // offset between blocks (mzh*lsmy for the small kernels)
  __device__ __forceinline__ int base(int r) const {
    const int b = (int)f_blk.div((uint32_t)r);
    return b * blk_stride + (r - b * per_blk);
  }
};

// R2C along z of nrows real rows held as packed pairs Z[j][lsz] in *a (row 2j in
// .x, row 2j+1 in .y): FFT each pair, then split into the half spectra written to
// X[rc.base(row) + q * rc.qstride], q in [0, nz/2].  Returns the buffer holding X.
__device__ float2* r2c_rows(float2* a, float2* b, const float2* twz, int nrows, int nz, int nzh,
                            int npairs, const RowCols& rc, const FastDiv& f_nzh) {
  const int lsz = pad_odd(nz);
  float2* Z = fft_lines<-1>(a, b, twz, nz, npairs, lsz);
  float2* X = (Z == a) ? b : a;
  const int items = npairs * nzh;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int j = (int)f_nzh.div((uint32_t)it), q = it - j * nzh;
    const float2 zq = Z[j * lsz + q];
    const float2 zm = Z[j * lsz + (q == 0 ? 0 : nz - q)];
    // A = (Z(q) + conj Z(-q))/2 ; B = (Z(q) - conj Z(-q))/(2i)
    X[rc.base(2 * j) + q * rc.qstride] = make_float2(0.5f * (zq.x + zm.x), 0.5f * (zq.y - zm.y));
    if (2 * j + 1 < nrows)
      X[rc.base(2 * j + 1) + q * rc.qstride] = make_float2(0.5f * (zq.y + zm.y), -0.5f * (zq.x - zm.x));
  }
  __syncthreads();
  return X;
}

// C2R along z: half spectra X[rc.base(row) + q * rc.qstride] in *a -> packed pairs
// Z[j][lsz] (Z = A + iB with the Hermitian extension), inverse FFT.  The imaginary
// parts of the q = 0 and q = nz/2 bins are dropped (they vanish for a Hermitian
// input).  Returns the buffer holding the packed real rows.
__device__ float2* c2r_rows(float2* a, float2* b, const float2* twz, int nrows, int nz, int npairs,
                            const RowCols& rc, const FastDiv& f_nz) {
  const int lsz = pad_odd(nz);
  const int items = npairs * nz;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int j = (int)f_nz.div((uint32_t)it), q = it - j * nz;
    const bool up = 2 * q > nz;
    const int qq = up ? nz - q : q;
    float2 x = a[rc.base(2 * j) + qq * rc.qstride];
    float2 y = (2 * j + 1 < nrows) ? a[rc.base(2 * j + 1) + qq * rc.qstride] : make_float2(0.f, 0.f);
    if (qq == 0 || 2 * qq == nz) { x.y = 0.f; y.y = 0.f; }
    if (up) { x.y = -x.y; y.y = -y.y; }
    b[j * lsz + q] = make_float2(x.x - y.y, x.y + y.x);      // x + i y
  }
  return fft_lines<+1>(b, a, twz, nz, npairs, lsz);
}

// c2r_rows restricted to the row pairs [j0, j1): pair j lands at line j - j0.
__device__ float2* c2r_rows_range(float2* a, float2* b, const float2* twz, int nrows, int nz, int j0, int j1,
                                  const RowCols& rc, const FastDiv& f_nz) {
  const int lsz = pad_odd(nz);
  const int items = (j1 - j0) * nz;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int jl = (int)f_nz.div((uint32_t)it), q = it - jl * nz;
    const int j = j0 + jl;
    const bool up = 2 * q > nz;
    const int qq = up ? nz - q : q;
    float2 x = a[rc.base(2 * j) + qq * rc.qstride];
    float2 y = (2 * j + 1 < nrows) ? a[rc.base(2 * j + 1) + qq * rc.qstride] : make_float2(0.f, 0.f);
    if (qq == 0 || 2 * qq == nz) { x.y = 0.f; y.y = 0.f; }
    if (up) { x.y = -x.y; y.y = -y.y; }
    b[jl * lsz + q] = make_float2(x.x - y.y, x.y + y.x);      // x + i y
  }
  return fft_lines<+1>(b, a, twz, nz, j1 - j0, lsz);
}

__device__ __forceinline__ RowCols plane_rowcols(const Geo& g) {
  RowCols rc;
  rc.qstride = g.lsy;
  rc.per_blk = g.ny;
  rc.f_blk = g.f_ny;
  rc.blk_stride = 0;
  return rc;
}

// Forward pass 1.  ps blocks per x-plane and component (vector model).  SRC_FISTA_Y
// reads y^k of the volume (a ignored) and is skipped once the volume's solve is done.
// LDS: tables (nz + ny) + two buffers of plane_lds complex.
template <int SRC>
__device__ __forceinline__ void plane_fwd_body(const VolDesc& vd, int lb, const float* __restrict__ a) {
  const Geo& g = vd.g;
  extern __shared__ float2 lds[];
  const int pl = plane_lds(g);
  float2* twz = lds;
  float2* twy = twz + g.nz;
  float2* P0 = twy + g.ny;
  float2* P1 = P0 + pl;
  // vector model: component comp of the plane is a workgroup of its own (components
  // outermost; a raw source has one)
  const int per_comp = g.ps * g.nx;
  const int comp = (SRC == SRC_RAW) ? 0 : lb / per_comp;
  lb -= comp * per_comp;
  // ps workgroups per plane: all of them transform every row along z, workgroup h
  // then takes the y-transforms of the columns qz in [q0, q1)
  const int h = lb / g.nx;
  const int x = plane_of_block(lb - h * g.nx, g.nx);
  const int q0 = h * g.nzh / g.ps, q1 = (h + 1) * g.nzh / g.ps;
  load_table(twz, vd.tw + vd.off[2], g.nz);
  load_table(twy, vd.tw + vd.off[1], g.ny);
  float c = 1.f;
  if constexpr (SRC == SRC_SCALED) c = (float)vd.st->scale;
  const long long pbase = (long long)x * g.ny * g.nz;
  const int nyz = g.ny * g.nz;
  const int lsz = pad_odd(g.nz);
  float* Zf = reinterpret_cast<float*>(P0);
  const float* __restrict__ b = vd.b + (long long)comp * g.N;
  batched<8, float>(nyz, [&](int p) { return plane_source<SRC>(pbase + p, a, nullptr, b, c); },
                    [&](int p, float v) {
                      const int y = (int)g.f_nz.div((uint32_t)p), z = p - y * g.nz;
                      Zf[2 * ((y >> 1) * lsz + z) + (y & 1)] = v;
                    });
  if (g.ny & 1) {
    for (int z = threadIdx.x; z < g.nz; z += blockDim.x) Zf[2 * ((g.ny >> 1) * lsz + z) + 1] = 0.f;
  }
  const RowCols rc = plane_rowcols(g);
  float2* X = r2c_rows(P0, P1, twz, g.ny, g.nz, g.nzh, g.npairs, rc, g.f_nzh);   // X[qz][lsy]
  // column qz of the result at Y[(qz - q0) * lsy]
  float2* Y = fft_lines<-1>(X + q0 * g.lsy, (X == P0 ? P1 : P0) + q0 * g.lsy, twy, g.ny, q1 - q0, g.lsy);
  float2* dst = vd.uperm + (long long)comp * g.hsz + (long long)x * g.plane;
  for (int e = threadIdx.x; e < g.plane; e += blockDim.x) {
    const int cc = (int)g.f_nmem.div((uint32_t)e), m = e - cc * g.nmem;
    const int cy = (int)g.f_mzh.div((uint32_t)cc), cz = cc - cy * g.mzh;
    const int jy = (int)g.f_sz.div((uint32_t)m), jz = m - jy * g.sz;
    const int qy = cy + jy * g.my, qz = cz + jz * g.mz;
    const bool direct = 2 * qz <= g.nz;
    const int col = direct ? qz : g.nz - qz;
    if (col < q0 || col >= q1) continue;
    float2 v;
    if (direct) {
      v = Y[(col - q0) * g.lsy + qy];
    } else {
      v = Y[(col - q0) * g.lsy + (qy == 0 ? 0 : g.ny - qy)];
      v.y = -v.y;
    }
    dst[e] = v;
  }
}
template <int SRC>
__global__ __launch_bounds__(1024) void k_plane_fwd(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                    const float* __restrict__ a) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  if constexpr (SRC == SRC_FISTA_Y || SRC == SRC_SCALED) {
    if (vd.st->done) return;
  }
  if constexpr (SRC == SRC_FISTA_Y) a = vd.y[vd.st->k & 1];
  if constexpr (SRC == SRC_SCALED) {
    if (!a) a = vd.rho[vd.st->k & 1];
  }
  plane_fwd_body<SRC>(vd, lb, a);
}

// ============================================================================ pass 2: classes
// HC = 0: compact spectra (one float per element; harmonic k is real if bit k of
// imag_mask is clear, purely imaginary if set).  HC = 1: complex spectra.
template <int HC, int E>
struct HLoad;

// Compact spectra: one float per element.
template <int E>
struct HLoad<0, E> {
  float v[E];
  __device__ __forceinline__ void load(const void* base, long long off) {
    const float* p = reinterpret_cast<const float*>(base) + off;
    if constexpr (E % 4 == 0) {
#pragma unroll
      for (int i = 0; i < E; i += 4) {
        const float4 t = *reinterpret_cast<const float4*>(p + i);
        v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
      }
    } else if constexpr (E % 2 == 0) {
#pragma unroll
      for (int i = 0; i < E; i += 2) {
        const float2 t = *reinterpret_cast<const float2*>(p + i);
        v[i] = t.x; v[i + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = p[i];
    }
  }
  __device__ __forceinline__ float re(int i) const { return v[i]; }
};

// Complex spectra.
template <int E>
struct HLoad<1, E> {
  float2 v[E];
  __device__ __forceinline__ void load(const void* base, long long off) {
    const float2* p = reinterpret_cast<const float2*>(base) + off;
    if constexpr (E % 2 == 0) {
#pragma unroll
      for (int i = 0; i < E; i += 2) {
        const float4 t = *reinterpret_cast<const float4*>(p + i);
        v[i] = make_float2(t.x, t.y); v[i + 1] = make_float2(t.z, t.w);
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = p[i];
    }
  }
};

// Destination of the forward class pass's decimated spectra F_k (the small-grid spectra
// of the portraits, before their inverse transform):
//   FWD_G          G = F  (the small-grid pass turns them into portraits)
//   FWD_ADJ        G' = my mz F (the adjoint takes them as they are: normal operator)
//   FWD_G_AND_ADJ  both (A then A^T: the portraits are written and A^T starts at once)
//   FWD_RESID      G' = my mz F - G, G holding the (unnormalised) small-grid spectra of
//                  the measured portraits (the solver's residual)
// Without boundary padding the small-grid inverse and forward transforms between the
// forward and the adjoint are, up to their scale my mz and to rounding, an identity on
// these spectra (they only make the two self-conjugate columns of each spectrum
// Hermitian, which F already is in exact arithmetic), so the adjoint can start from F.
// With padding the crop to the field of view sits between them and the pass stays.
enum { FWD_G = 0, FWD_ADJ = 1, FWD_G_AND_ADJ = 2, FWD_RESID = 3 };

// LDS layout of the class kernels: tables (nx + mx), U0/U1 (W lines of lsx, the
// x-transforms of the W = cpw*nmem member columns), F0/F1 (K*cpw lines of mx).
__host__ __device__ inline size_t class_lds_elems(const Geo& g) {
  const size_t W = (size_t)g.cpw * g.nmem;
  return (size_t)g.nx + g.mx + 2 * W * g.lsx + 2 * (size_t)g.K * g.cpw * g.mx;
}

// Harmonics of spectra prefetched ahead in the class kernels: 8 for compact spectra
// with up to 4 elements per thread (the whole ring costs <= 32 registers), else 4.
__host__ __device__ constexpr int hpf_of(int HC, int E) { return (HC == 0 && E <= 4) ? 8 : 4; }

// Position of class-layout element p of a (k, x'-block, class, x'-in-block) store,
// p over K*cpw*mx, as offsets into F ((k*cpw + c)*mx + x') and G.
__device__ __forceinline__ void class_g_index(const Geo& g, int p, int c0, int& fo, long long& go) {
  const int k = (int)g.f_cpwmx.div((uint32_t)p), r = p - k * g.cpw * g.mx;
  const int xbi = (int)g.f_cpwxb.div((uint32_t)r), r2 = r - xbi * g.cpw * g.xb;
  const int c = (int)g.f_xb.div((uint32_t)r2), xi = r2 - c * g.xb;
  const int nxb = g.mx / g.xb;
  fo = (k * g.cpw + c) * g.mx + xbi * g.xb + xi;
  go = (((long long)k * nxb + xbi) * g.ncls + c0 + c) * g.xb + xi;
}

// Forward pass 2 of one block (cpw classes).  Threads beyond vd.T_class only take
// part in the barriers and shuffles (batched launches use the largest block size).
// VEC: vector model, vd.ncomp components (else one, and the loop folds away).
// mode (FWD_*) selects where the decimated spectra go.
template <int HC, int E, bool VEC = false>
__device__ __forceinline__ void class_fwd_body(const VolDesc& vd, int lb, int mode) {
  constexpr int HPF = hpf_of(HC, E);
  const Geo& g = vd.g;
  extern __shared__ float2 lds[];
  const int W = g.cpw * g.nmem;
  float2* twx = lds;
  float2* twm = twx + g.nx;
  float2* U0 = twm + g.mx;
  float2* U1 = U0 + W * g.lsx;
  float2* F0 = U1 + W * g.lsx;
  float2* F1 = F0 + g.K * g.cpw * g.mx;
  const int c0 = lb * g.cpw;
  const bool act = (int)threadIdx.x < vd.T_class;
  // this thread's E spectrum elements: all share class cl and folded frequency qxp
  const int e0 = act ? (int)threadIdx.x * E : 0;
  const int per_cls = g.mx * g.S;
  const int cl = (int)g.f_mxS.div((uint32_t)e0);
  const int rem = e0 - cl * per_cls;
  const int qxp = (int)g.f_S.div((uint32_t)rem);
  const int within = rem - qxp * g.S;
  const void* hs = vd.hs;
  const int LG = g.S / E;
  const uint32_t imag_mask = vd.imag_mask;
  // vector model: the products of every component accumulate in F0 before the one
  // inverse transform (the sum over i commutes with it)
  const int ncomp = VEC ? vd.ncomp : 1;
  uint32_t before = 0;   // harmonics some earlier component has written to F0
  for (int comp = 0; comp < ncomp; ++comp) {
  if (comp) __syncthreads();   // the previous component's U is still being read
  const uint32_t pm = VEC ? vd.cmask[comp] : ~0u;
  const long long hoff0 = (long long)c0 * per_cls + e0 + comp * vd.hs_cstride;
  // spectra do not depend on the data: start streaming them first
  HLoad<HC, E> hb[HPF];
#pragma unroll
  for (int i = 0; i < HPF; ++i)
    if (act && i < g.K && ((pm >> i) & 1u)) hb[i].load(hs, (long long)i * g.hsz + hoff0);
  if (comp == 0) {
    load_table(twx, vd.tw + vd.off[0], g.nx);
    load_table(twm, vd.tw + vd.off[3], g.mx);
  }
  const float2* __restrict__ uperm = vd.uperm + (long long)comp * g.hsz;
  batched<8, float2>(g.nx * W,
                     [&](int p) {
                       const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
                       return uperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e];
                     },
                     [&](int p, float2 v) {
                       const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
                       U0[e * g.lsx + xx] = v;
                     });
  const float2* U = fft_lines<-1>(U0, U1, twx, g.nx, W, g.lsx);
  float2 ur[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int w = within + i;
    const int jx = (int)g.f_nmem.div((uint32_t)w), m = w - jx * g.nmem;
    ur[i] = act ? U[(cl * g.nmem + m) * g.lsx + qxp + jx * g.mx] : make_float2(0.f, 0.f);
  }
  for (int k0 = 0; k0 < g.K; k0 += HPF) {
#pragma unroll
    for (int i = 0; i < HPF; ++i) {
      const int k = k0 + i;
      if (k < g.K) {
        // pk is the same for the whole block (it depends on k and the component only)
        const bool pk = ((pm >> k) & 1u) != 0;
        float2 acc = make_float2(0.f, 0.f);
        if (act) {
          if (pk) {
            if constexpr (HC == 0) {
#pragma unroll
              for (int t = 0; t < E; ++t) { acc.x += hb[i].v[t] * ur[t].x; acc.y += hb[i].v[t] * ur[t].y; }
              if ((imag_mask >> k) & 1u) acc = make_float2(-acc.y, acc.x);
            } else {
#pragma unroll
              for (int t = 0; t < E; ++t) acc = cadd(acc, cmul(hb[i].v[t], ur[t]));
            }
          }
          if (k + HPF < g.K && ((pm >> (k + HPF)) & 1u)) hb[i].load(hs, (long long)(k + HPF) * g.hsz + hoff0);
        }
        if (pk) {
          for (int o = LG >> 1; o >= 1; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o, 64);
            acc.y += __shfl_xor(acc.y, o, 64);
          }
          if (act && (threadIdx.x & (LG - 1)) == 0) {
            float2& f = F0[(k * g.cpw + cl) * g.mx + qxp];
            f = ((before >> k) & 1u) ? cadd(f, acc) : acc;
          }
        }
      }
    }
  }
  before |= pm;
  }
  const float2* F = fft_lines<+1>(F0, F1, twm, g.mx, g.K * g.cpw, g.mx);
  float2* __restrict__ G = vd.G;
  float2* __restrict__ Gp = vd.Gp;
  // the small-grid transforms are unnormalised: their round trip scales by my mz
  const float syz = (float)(g.my * g.mz);
  for (int p = threadIdx.x; p < g.K * g.cpw * g.mx; p += blockDim.x) {
    int fo;
    long long go;
    class_g_index(g, p, c0, fo, go);
    const float2 f = F[fo];
    if (mode == FWD_G || mode == FWD_G_AND_ADJ) G[go] = f;
    if (mode == FWD_ADJ || mode == FWD_G_AND_ADJ) Gp[go] = make_float2(syz * f.x, syz * f.y);
    if (mode == FWD_RESID) {
      const float2 dh = G[go];
      Gp[go] = make_float2(syz * f.x - dh.x, syz * f.y - dh.y);
    }
  }
}

// Adjoint pass 2 of one block.
template <int HC, int E, bool VEC = false>
__device__ __forceinline__ void class_adj_body(const VolDesc& vd, int lb) {
  constexpr int HPF = hpf_of(HC, E);
  const Geo& g = vd.g;
  extern __shared__ float2 lds[];
  const int W = g.cpw * g.nmem;
  float2* twx = lds;
  float2* twm = twx + g.nx;
  float2* U0 = twm + g.mx;
  float2* U1 = U0 + W * g.lsx;
  float2* F0 = U1 + W * g.lsx;
  float2* F1 = F0 + g.K * g.cpw * g.mx;
  const int c0 = lb * g.cpw;
  const bool act = (int)threadIdx.x < vd.T_class;
  const int e0 = act ? (int)threadIdx.x * E : 0;
  const int per_cls = g.mx * g.S;
  const int cl = (int)g.f_mxS.div((uint32_t)e0);
  const int rem = e0 - cl * per_cls;
  const int qxp = (int)g.f_S.div((uint32_t)rem);
  const int within = rem - qxp * g.S;
  const void* hs = vd.hs;
  HLoad<HC, E> hb[HPF];
  const uint32_t pm0 = VEC ? vd.cmask[0] : ~0u;
#pragma unroll
  for (int i = 0; i < HPF; ++i)
    if (act && i < g.K && ((pm0 >> i) & 1u)) hb[i].load(hs, (long long)i * g.hsz + (long long)c0 * per_cls + e0);
  load_table(twx, vd.tw + vd.off[0], g.nx);
  load_table(twm, vd.tw + vd.off[3], g.mx);
  const float2* __restrict__ Gp = vd.Gp;
  batched<8, float2>(g.K * g.cpw * g.mx,
                     [&](int p) {
                       int fo;
                       long long go;
                       class_g_index(g, p, c0, fo, go);
                       return Gp[go];
                     },
                     [&](int p, float2 v) {
                       int fo;
                       long long go;
                       class_g_index(g, p, c0, fo, go);
                       F0[fo] = v;
                     });
  const float2* F = fft_lines<-1>(F0, F1, twm, g.mx, g.K * g.cpw, g.mx);
  // vector model: H_{k,i}^T of every component i from the one transform of the data
  const int ncomp = VEC ? vd.ncomp : 1;
  for (int comp = 0; comp < ncomp; ++comp) {
  const long long hoff0 = (long long)c0 * per_cls + e0 + comp * vd.hs_cstride;
  const uint32_t pm = VEC ? vd.cmask[comp] : ~0u;
  if (comp) {
    __syncthreads();   // the previous component's store still reads U0/U1
#pragma unroll
    for (int i = 0; i < HPF; ++i)
      if (act && i < g.K && ((pm >> i) & 1u)) hb[i].load(hs, (long long)i * g.hsz + hoff0);
  }
  float2 acc[E];
#pragma unroll
  for (int t = 0; t < E; ++t) acc[t] = make_float2(0.f, 0.f);
  const uint32_t imag_mask = vd.imag_mask;
  for (int k0 = 0; k0 < g.K; k0 += HPF) {
#pragma unroll
    for (int i = 0; i < HPF; ++i) {
      const int k = k0 + i;
      if (act && k < g.K) {
        if ((pm >> k) & 1u) {
          float2 R = F[(k * g.cpw + cl) * g.mx + qxp];
          if constexpr (HC == 0) {
            // conj(i h) R = -i h R
            if ((imag_mask >> k) & 1u) R = make_float2(R.y, -R.x);
#pragma unroll
            for (int t = 0; t < E; ++t) { acc[t].x += hb[i].v[t] * R.x; acc[t].y += hb[i].v[t] * R.y; }
          } else {
#pragma unroll
            for (int t = 0; t < E; ++t) acc[t] = cadd(acc[t], cmulcj(hb[i].v[t], R));
          }
        }
        if (k + HPF < g.K && ((pm >> (k + HPF)) & 1u)) hb[i].load(hs, (long long)(k + HPF) * g.hsz + hoff0);
      }
    }
  }
  // every element of the group is written exactly once
  if (act) {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int w = within + t;
      const int jx = (int)g.f_nmem.div((uint32_t)w), m = w - jx * g.nmem;
      U0[(cl * g.nmem + m) * g.lsx + qxp + jx * g.mx] = acc[t];
    }
  }
  const float2* V = fft_lines<+1>(U0, U1, twx, g.nx, W, g.lsx);
  float2* __restrict__ vperm = vd.uperm + (long long)comp * g.hsz;
  for (int p = threadIdx.x; p < g.nx * W; p += blockDim.x) {
    const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
    vperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e] = V[e * g.lsx + xx];
  }
  }
}

// Forward and adjoint class passes in one (scalar model, no boundary padding), for the
// solver's updates, the normal operator and A then A^T.  The folded spectra Fhat_k of
// the block's classes (class_fwd_body's F0, before its inverse x' transform) stay in
// LDS, and the adjoint starts from them: the inverse x' transform, the small-grid
// inverse and forward transforms and the forward x' transform between the two passes
// compose to multiplication by M = mx my mz (up to rounding), so the adjoint's decimated
// spectra are
//   NRM_RESID  R_k = M Fhat_k - Dt_k, Dt = the x' transform of the measured portraits'
//              small-grid spectra (k_class_data, in G' as [k][class][qx'])
//   NRM_PLAIN  R_k = M Fhat_k                       (normal operator)
//   NRM_STORE  R_k = M Fhat_k, and G = the inverse x' transform of Fhat (the small-grid
//              pass turns it into the portraits)
// Each spectrum Hhat_k is read from HBM once: with K at most the prefetch ring's depth the
// ring still holds all of them for the adjoint, else the adjoint's second read is of the
// block's own recently read spectra (L2).
enum { NRM_RESID = 0, NRM_PLAIN = 1, NRM_STORE = 2 };

// The fused pass keeps every harmonic's spectra of its elements in registers when they
// fit (compact spectra, K <= 12 at E <= 4): all loads are issued at the start and the
// adjoint reuses them, so the pass waits on one round of spectrum loads.
__host__ __device__ constexpr int hpf_normal(int HC, int E) { return (HC == 0 && E <= 4) ? 12 : hpf_of(HC, E); }

template <int HC, int E>
__device__ __forceinline__ void class_normal_body(const VolDesc& vd, int lb, int mode) {
  constexpr int HPF = hpf_normal(HC, E);
  const Geo& g = vd.g;
  extern __shared__ float2 lds[];
  const int W = g.cpw * g.nmem;
  float2* twx = lds;
  float2* twm = twx + g.nx;
  float2* U0 = twm + g.mx;
  float2* U1 = U0 + W * g.lsx;
  float2* F0 = U1 + W * g.lsx;
  float2* F1 = F0 + g.K * g.cpw * g.mx;
  const int c0 = lb * g.cpw;
  const bool act = (int)threadIdx.x < vd.T_class;
  const int e0 = act ? (int)threadIdx.x * E : 0;
  const int per_cls = g.mx * g.S;
  const int cl = (int)g.f_mxS.div((uint32_t)e0);
  const int rem = e0 - cl * per_cls;
  const int qxp = (int)g.f_S.div((uint32_t)rem);
  const int within = rem - qxp * g.S;
  const long long hoff0 = (long long)c0 * per_cls + e0;
  const void* hs = vd.hs;
  const int LG = g.S / E;
  const uint32_t imag_mask = vd.imag_mask;
  const int KCM = g.K * g.cpw * g.mx;
  HLoad<HC, E> hb[HPF];
  // a ring that holds every harmonic is loaded after the x transform (its registers
  // would otherwise be live across it); a shorter ring starts streaming at once
  constexpr bool kLate = HPF > hpf_of(HC, E);
  if constexpr (!kLate) {
#pragma unroll
    for (int i = 0; i < HPF; ++i)
      if (act && i < g.K) hb[i].load(hs, (long long)i * g.hsz + hoff0);
  }
  // the data term of the block's classes (F1[(k cpw + c) mx + qx'])
  if (mode == NRM_RESID) {
    const float2* __restrict__ Dt = vd.Gp;
    batched<8, float2>(KCM,
                       [&](int p) {
                         const int k = (int)g.f_cpwmx.div((uint32_t)p), r = p - k * g.cpw * g.mx;
                         const int c = r / g.mx, q = r - c * g.mx;
                         return Dt[((long long)k * g.ncls + c0 + c) * g.mx + q];
                       },
                       [&](int p, float2 v) { F1[p] = v; });
  }
  load_table(twx, vd.tw + vd.off[0], g.nx);
  load_table(twm, vd.tw + vd.off[3], g.mx);
  const float2* __restrict__ uperm = vd.uperm;
  batched<8, float2>(g.nx * W,
                     [&](int p) {
                       const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
                       return uperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e];
                     },
                     [&](int p, float2 v) {
                       const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
                       U0[e * g.lsx + xx] = v;
                     });
  const float2* U = fft_lines<-1>(U0, U1, twx, g.nx, W, g.lsx);
  float2 ur[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int w = within + i;
    const int jx = (int)g.f_nmem.div((uint32_t)w), m = w - jx * g.nmem;
    ur[i] = act ? U[(cl * g.nmem + m) * g.lsx + qxp + jx * g.mx] : make_float2(0.f, 0.f);
  }
  if constexpr (kLate) {
#pragma unroll
    for (int i = 0; i < HPF; ++i)
      if (act && i < g.K) hb[i].load(hs, (long long)i * g.hsz + hoff0);
  }
  // forward: Fhat_k(cl, qx') = sum over the S alias members of Hhat_k U
  for (int k0 = 0; k0 < g.K; k0 += HPF) {
#pragma unroll
    for (int i = 0; i < HPF; ++i) {
      const int k = k0 + i;
      if (k < g.K) {
        float2 acc = make_float2(0.f, 0.f);
        if (act) {
          if constexpr (HC == 0) {
#pragma unroll
            for (int t = 0; t < E; ++t) { acc.x += hb[i].v[t] * ur[t].x; acc.y += hb[i].v[t] * ur[t].y; }
            if ((imag_mask >> k) & 1u) acc = make_float2(-acc.y, acc.x);
          } else {
#pragma unroll
            for (int t = 0; t < E; ++t) acc = cadd(acc, cmul(hb[i].v[t], ur[t]));
          }
          if (k + HPF < g.K) hb[i].load(hs, (long long)(k + HPF) * g.hsz + hoff0);
        }
        for (int o = LG >> 1; o >= 1; o >>= 1) {
          acc.x += __shfl_xor(acc.x, o, 64);
          acc.y += __shfl_xor(acc.y, o, 64);
        }
        if (act && (threadIdx.x & (LG - 1)) == 0) F0[(k * g.cpw + cl) * g.mx + qxp] = acc;
      }
    }
  }
  __syncthreads();   // Fhat complete; U0/U1 free for the adjoint
  // adjoint: sum_k conj(Hhat_k) R_k for each alias member, then the inverse x transform.
  // With K <= HPF the ring still holds every harmonic's spectra.
  if (g.K > HPF) {
#pragma unroll
    for (int i = 0; i < HPF; ++i)
      if (act) hb[i].load(hs, (long long)i * g.hsz + hoff0);
  }
  const float Mf = (float)g.M;
  float2 acc[E];
#pragma unroll
  for (int t = 0; t < E; ++t) acc[t] = make_float2(0.f, 0.f);
  for (int k0 = 0; k0 < g.K; k0 += HPF) {
#pragma unroll
    for (int i = 0; i < HPF; ++i) {
      const int k = k0 + i;
      if (act && k < g.K) {
        const int fi = (k * g.cpw + cl) * g.mx + qxp;
        const float2 f = F0[fi];
        float2 R = make_float2(Mf * f.x, Mf * f.y);
        if (mode == NRM_RESID) R = csub(R, F1[fi]);
        if constexpr (HC == 0) {
          // conj(i h) R = -i h R
          if ((imag_mask >> k) & 1u) R = make_float2(R.y, -R.x);
#pragma unroll
          for (int t = 0; t < E; ++t) { acc[t].x += hb[i].v[t] * R.x; acc[t].y += hb[i].v[t] * R.y; }
        } else {
#pragma unroll
          for (int t = 0; t < E; ++t) acc[t] = cadd(acc[t], cmulcj(hb[i].v[t], R));
        }
        if (k + HPF < g.K) hb[i].load(hs, (long long)(k + HPF) * g.hsz + hoff0);
      }
    }
  }
  if (act) {
#pragma unroll
    for (int t = 0; t < E; ++t) {
      const int w = within + t;
      const int jx = (int)g.f_nmem.div((uint32_t)w), m = w - jx * g.nmem;
      U0[(cl * g.nmem + m) * g.lsx + qxp + jx * g.mx] = acc[t];
    }
  }
  const float2* V = fft_lines<+1>(U0, U1, twx, g.nx, W, g.lsx);
  float2* __restrict__ vperm = vd.uperm;
  for (int p = threadIdx.x; p < g.nx * W; p += blockDim.x) {
    const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
    vperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e] = V[e * g.lsx + xx];
  }
  if (mode == NRM_STORE) {
    // the portraits' small-grid spectra, as class_fwd_body writes them (F0 still holds
    // Fhat: the adjoint only read it)
    const float2* F = fft_lines<+1>(F0, F1, twm, g.mx, g.K * g.cpw, g.mx);
    float2* __restrict__ G = vd.G;
    for (int p = threadIdx.x; p < KCM; p += blockDim.x) {
      int fo;
      long long go;
      class_g_index(g, p, c0, fo, go);
      G[go] = F[fo];
    }
  }
}

// Dt = the x' transform of the measured portraits' small-grid spectra (G, as k_small_fwd
// left them), into G' as [k][class][qx'], for class_normal_body's residual.  Same
// blocks and LDS layout as the class passes.
__global__ __launch_bounds__(1024) void k_class_data(const VolDesc* __restrict__ vds) {
  const VolDesc& vd = vds[0];
  const Geo& g = vd.g;
  const int lb = blockIdx.x;
  extern __shared__ float2 lds[];
  const int W = g.cpw * g.nmem;
  float2* twm = lds + g.nx;
  float2* F0 = twm + g.mx + 2 * W * g.lsx;
  float2* F1 = F0 + g.K * g.cpw * g.mx;
  const int c0 = lb * g.cpw;
  const int KCM = g.K * g.cpw * g.mx;
  load_table(twm, vd.tw + vd.off[3], g.mx);
  const float2* __restrict__ Dh = vd.G;
  batched<8, float2>(KCM,
                     [&](int p) {
                       int fo;
                       long long go;
                       class_g_index(g, p, c0, fo, go);
                       return Dh[go];
                     },
                     [&](int p, float2 v) {
                       int fo;
                       long long go;
                       class_g_index(g, p, c0, fo, go);
                       F0[fo] = v;
                     });
  const float2* F = fft_lines<-1>(F0, F1, twm, g.mx, g.K * g.cpw, g.mx);
  float2* __restrict__ Dt = vd.Gp;
  for (int p = threadIdx.x; p < KCM; p += blockDim.x) {
    const int k = (int)g.f_cpwmx.div((uint32_t)p), r = p - k * g.cpw * g.mx;
    const int c = r / g.mx, q = r - c * g.mx;
    Dt[((long long)k * g.ncls + c0 + c) * g.mx + q] = F[p];
  }
}

// Single-volume class passes, grid = ncls/cpw blocks of T_class threads.
// check_done skips the launch once the volume's solve is done.
// XCD-aware: consecutive class blocks run on one XCD, so the short runs of G, G' and
// the class-layout spectra that neighbouring blocks share are fetched into one L2.
template <int HC, int E, bool VEC>
__global__ __launch_bounds__(1024) void k_class_fwd(const VolDesc* __restrict__ vds, int check_done, int mode) {
  int lb;
  const VolDesc& vd = vol_of(vds, nullptr, lb);
  if (check_done && vd.st->done) return;
  class_fwd_body<HC, E, VEC>(vd, plane_of_block(lb, gridDim.x), mode);
}
template <int HC, int E>
__global__ __launch_bounds__(1024) void k_class_normal(const VolDesc* __restrict__ vds, int check_done, int mode) {
  int lb;
  const VolDesc& vd = vol_of(vds, nullptr, lb);
  if (check_done && vd.st->done) return;
  class_normal_body<HC, E>(vd, plane_of_block(lb, gridDim.x), mode);
}
template <int HC, int E, bool VEC>
__global__ __launch_bounds__(1024) void k_class_adj(const VolDesc* __restrict__ vds, int check_done) {
  int lb;
  const VolDesc& vd = vol_of(vds, nullptr, lb);
  if (check_done && vd.st->done) return;
  class_adj_body<HC, E, VEC>(vd, plane_of_block(lb, gridDim.x));
}

// Batched class passes over a task table (compact spectra), the element split E
// of each volume dispatched per block.  Volumes whose solve is done are skipped.
#define MH3D_E_SWITCH(BODY, ...)                         \
  switch (vd.g.E) {                                      \
    case 8: BODY<0, 8>(vd, lb __VA_ARGS__); break;       \
    case 6: BODY<0, 6>(vd, lb __VA_ARGS__); break;       \
    case 4: BODY<0, 4>(vd, lb __VA_ARGS__); break;       \
    case 3: BODY<0, 3>(vd, lb __VA_ARGS__); break;       \
    case 2: BODY<0, 2>(vd, lb __VA_ARGS__); break;       \
    case 9: BODY<0, 9>(vd, lb __VA_ARGS__); break;       \
    default: BODY<0, 1>(vd, lb __VA_ARGS__); break;      \
  }
// Padded volumes of a batch (mode FWD_G: their small-grid pass crops to the field of view).
__global__ __launch_bounds__(1024) void k_class_fwd_batch(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                          int mode) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  if (vd.st->done) return;
  MH3D_E_SWITCH(class_fwd_body, , mode)
}
// mode: NRM_RESID (solver) or NRM_PLAIN (power iteration); volumes without padding.
__global__ __launch_bounds__(1024) void k_class_normal_batch(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                             int mode) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  if (vd.st->done) return;
  MH3D_E_SWITCH(class_normal_body, , mode)
}
__global__ __launch_bounds__(1024) void k_class_adj_batch(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  if (vd.st->done) return;
  MH3D_E_SWITCH(class_adj_body, )
}
#undef MH3D_E_SWITCH

// ============================================================================ pass 3: small grid
enum { EPI_STORE = 0, EPI_RESID = 1, EPI_RESID_BACK = 2, EPI_BACK = 3, EPI_STORE_BACK = 4 };

// Small-grid LDS layout: column (xi, q'z) holds the y' line at
// X[(xi*mzh + q'z)*lsmy + y'], rows r = xi*my + y' of real data are packed in pairs.
__device__ __forceinline__ RowCols small_rowcols(const Geo& g) {
  RowCols rc;
  rc.qstride = g.lsmy;
  rc.per_blk = g.my;
  rc.f_blk = g.f_my;
  rc.blk_stride = g.mzh * g.lsmy;
  return rc;
}

// 2-D R2C over (y', z') of the small-grid rows held as packed pairs in *a, then
// store the class layout G[k][xbi][class][xi].
__device__ void small_r2c_and_store(const Geo& g, float2* a, float2* b, const float2* twy, const float2* twz,
                                    float2* __restrict__ Gout, int k, int xbi) {
  const int rows = g.xb * g.my;
  float2* X = r2c_rows(a, b, twz, rows, g.mz, g.mzh, g.spairs, small_rowcols(g), g.f_mzh);
  float2* Y = fft_lines<-1>(X, X == a ? b : a, twy, g.my, g.xb * g.mzh, g.lsmy);
  const int nxb = g.mx / g.xb;
  float2* dst = Gout + ((long long)k * nxb + xbi) * g.ncls * g.xb;
  for (int p = threadIdx.x; p < g.ncls * g.xb; p += blockDim.x) {
    const int c = (int)g.f_xb.div((uint32_t)p), xi = p - c * g.xb;
    const int qy = (int)g.f_mzh.div((uint32_t)c), qz = c - qy * g.mzh;
    dst[p] = Y[(xi * g.mzh + qz) * g.lsmy + qy];
  }
}

// Portrait index of element p = (xi*my + y')*mz + z' of x'-block xbi, harmonic k, in
// the field-of-view portraits [K][mxf][myf][mzf]; -1 for a sample of the padding.
__device__ __forceinline__ long long fov_index(const Geo& g, int k, int xbi, int p) {
  const int r = (int)g.f_mz.div((uint32_t)p), z = p - r * g.mz;
  const int xi = (int)g.f_my.div((uint32_t)r), y = r - xi * g.my;
  const int xf = xbi * g.xb + xi - g.pxs, yf = y - g.pys, zf = z - g.pzs;
  if ((unsigned)xf >= (unsigned)g.mxf || (unsigned)yf >= (unsigned)g.myf || (unsigned)zf >= (unsigned)g.mzf) return -1;
  return (long long)k * g.Mf + ((long long)xf * g.myf + yf) * g.mzf + zf;
}

// Forward pass 3 (and, with EPI_RESID_BACK / EPI_BACK, the first adjoint pass on
// the result).  One block per (k, x'-block).  EPI_RESID_BACK uses the volume's data
// and is skipped once its solve is done.  LDS: tables (my + mz) + 2 * small_lds.
template <int EPI>
__device__ __forceinline__ void small_inv_body(const VolDesc& vd, int lb, float* __restrict__ d) {
  const Geo& g = vd.g;
  if constexpr (EPI == EPI_RESID_BACK || EPI == EPI_BACK) {
    if (vd.st->done) return;
  }
  const float* __restrict__ dmeas = vd.d;
  extern __shared__ float2 lds[];
  const int sl = small_lds(g);
  float2* twy = lds;
  float2* twz = twy + g.my;
  float2* P0 = twz + g.mz;
  float2* P1 = P0 + sl;
  load_table(twy, vd.tw + vd.off[4], g.my);
  load_table(twz, vd.tw + vd.off[5], g.mz);
  const int nxb = g.mx / g.xb;
  const int k = lb / nxb, xbi = lb - (lb / nxb) * nxb;
  const float2* src = vd.G + ((long long)k * nxb + xbi) * g.ncls * g.xb;
  batched<8, float2>(g.ncls * g.xb, [&](int p) { return src[p]; },
                     [&](int p, float2 v) {
                       const int c = (int)g.f_xb.div((uint32_t)p), xi = p - c * g.xb;
                       const int qy = (int)g.f_mzh.div((uint32_t)c), qz = c - qy * g.mzh;
                       P0[(xi * g.mzh + qz) * g.lsmy + qy] = v;
                     });
  float2* X = fft_lines<+1>(P0, P1, twy, g.my, g.xb * g.mzh, g.lsmy);
  const int rows = g.xb * g.my;
  float2* Z = c2r_rows(X, X == P0 ? P1 : P0, twz, rows, g.mz, g.spairs, small_rowcols(g), g.f_mz);
  // Z holds packed real rows: row r at pair r/2, .x (even) / .y (odd), line stride lsmz
  const int lsmz = pad_odd(g.mz);
  float* Zf = reinterpret_cast<float*>(Z);
  const long long obase = (long long)k * g.M + (long long)xbi * g.xb * g.my * g.mz;
  const int n = rows * g.mz;
  auto lidx = [&](int p) {
    const int r = (int)g.f_mz.div((uint32_t)p), z = p - r * g.mz;
    return 2 * ((r >> 1) * lsmz + z) + (r & 1);
  };
  if (g.padded) {
    // boundary padding: only the field-of-view samples are data (C P); the padding's
    // samples of the residual are zero (C^T C P)
    if constexpr (EPI == EPI_STORE || EPI == EPI_STORE_BACK) {
      for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const long long di = fov_index(g, k, xbi, p);
        const int li = lidx(p);
        if (di >= 0) d[di] = Zf[li];
        else if (EPI == EPI_STORE_BACK) Zf[li] = 0.f;
      }
    } else if constexpr (EPI == EPI_RESID) {
      for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const long long di = fov_index(g, k, xbi, p);
        if (di >= 0) d[di] = Zf[lidx(p)] - dmeas[di];
      }
    } else if constexpr (EPI == EPI_RESID_BACK) {
      for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const long long di = fov_index(g, k, xbi, p);
        const int li = lidx(p);
        Zf[li] = di >= 0 ? Zf[li] - dmeas[di] : 0.f;
      }
    } else if constexpr (EPI == EPI_BACK) {
      for (int p = threadIdx.x; p < n; p += blockDim.x)
        if (fov_index(g, k, xbi, p) < 0) Zf[lidx(p)] = 0.f;
    }
  } else if constexpr (EPI == EPI_STORE || EPI == EPI_STORE_BACK) {
    for (int p = threadIdx.x; p < n; p += blockDim.x) d[obase + p] = Zf[lidx(p)];
  } else if constexpr (EPI == EPI_RESID) {
    batched<8, float>(n, [&](int p) { return dmeas[obase + p]; },
                      [&](int p, float m) { d[obase + p] = Zf[lidx(p)] - m; });
  } else if constexpr (EPI == EPI_RESID_BACK) {
    batched<8, float>(n, [&](int p) { return dmeas[obase + p]; },
                      [&](int p, float m) { const int li = lidx(p); Zf[li] = Zf[li] - m; });
  }
  // EPI_BACK keeps the values in place; EPI_STORE_BACK stores them and transforms them back
  if constexpr (EPI == EPI_RESID_BACK || EPI == EPI_BACK || EPI == EPI_STORE_BACK) {
    if (rows & 1) {
      for (int z = threadIdx.x; z < g.mz; z += blockDim.x) Zf[2 * ((rows >> 1) * lsmz + z) + 1] = 0.f;
    }
    small_r2c_and_store(g, Z, Z == P0 ? P1 : P0, twy, twz, vd.Gp, k, xbi);
  }
}
template <int EPI>
__global__ __launch_bounds__(1024) void k_small_inv(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                    float* __restrict__ d) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  small_inv_body<EPI>(vd, lb, d);
}

// Adjoint pass 3: R2C of the portraits r.  One block per (k, x'-block).
// out: the spectra's destination (NULL: G').
__global__ __launch_bounds__(1024) void k_small_fwd(const VolDesc* __restrict__ vds, const float* __restrict__ r,
                                                   float2* __restrict__ out) {
  int lb;
  const VolDesc& vd = vol_of(vds, nullptr, lb);
  const Geo& g = vd.g;
  extern __shared__ float2 lds[];
  const int sl = small_lds(g);
  float2* twy = lds;
  float2* twz = twy + g.my;
  float2* P0 = twz + g.mz;
  float2* P1 = P0 + sl;
  load_table(twy, vd.tw + vd.off[4], g.my);
  load_table(twz, vd.tw + vd.off[5], g.mz);
  const int nxb = g.mx / g.xb;
  const int k = lb / nxb, xbi = lb - (lb / nxb) * nxb;
  const int rows = g.xb * g.my;
  const int lsmz = pad_odd(g.mz);
  const long long ibase = (long long)k * g.M + (long long)xbi * g.xb * g.my * g.mz;
  float* Zf = reinterpret_cast<float*>(P0);
  const int n = rows * g.mz;
  // with boundary padding the portraits cover the field of view: C^T r is zero outside
  batched<8, float>(n, [&](int p) {
                      if (!g.padded) return r[ibase + p];
                      const long long di = fov_index(g, k, xbi, p);
                      return di >= 0 ? r[di] : 0.f;
                    },
                    [&](int p, float v) {
                      const int rr = (int)g.f_mz.div((uint32_t)p), z = p - rr * g.mz;
                      Zf[2 * ((rr >> 1) * lsmz + z) + (rr & 1)] = v;
                    });
  if (rows & 1) {
    for (int z = threadIdx.x; z < g.mz; z += blockDim.x) Zf[2 * ((rows >> 1) * lsmz + z) + 1] = 0.f;
  }
  small_r2c_and_store(g, P0, P1, twy, twz, out ? out : vd.Gp, k, xbi);
}

// ============================================================================ pass 1 adjoint
enum { OUT_SCALE_B = 0, OUT_U = 1, OUT_STEP_NORMAL = 2, OUT_STEP_FISTA = 3 };
enum { UPD_NORMAL = 1, UPD_FISTA = 2 };

struct AdjOut {
  float* out;              // OUT_SCALE_B / UPD_NORMAL: result (UPD_NORMAL: NULL -> rho[(k+1) & 1])
  const float* yin;        // UPD_NORMAL: w_{t-1} (v = scale * w_{t-1}); NULL -> rho[k & 1]
};

// The 13 values of one voxel's regulariser stencil and the values its update reads.
struct StencilVals {
  float c, zm2, zm1, zp1, zp2, ym2, ym1, yp1, yp2, xm2, xm1, xp1, xp2, u, rk;
  bool shell;              // on the boundary prior's shell
};

// The voxel-wise end of a solver step, after the adjoint left u = b . v (the A^T A part):
//   UPD_NORMAL  out = u + lam T^T T (s w_prev); FP64 <s w_prev, out>, ||out||^2
//               (power iteration: lmax, next scale 1/||out||)
//   UPD_FISTA   g = u + lam T^T T y^k; rho^{k+1} = max(y^k - tau g, 0);
//               y^{k+1} = rho^{k+1} + k/(k+3) (rho^{k+1} - rho^k);
//               FP64 ||rho^{k+1} - y^k||^2, ||rho^{k+1}||^2, count of non-finite g
// T^T T is the periodic 13-point stencil sum_a (v[+2] - 4v[+1] + 6v - 4v[-1] + v[-2])
// of stacked second differences (reg_kind 1: T = I); neighbours are read from global
// memory (cache resident).  Used by k_vol_update and by the adjoint plane pass that
// finishes the step itself (OUT_STEP_*).
template <int UPD>
struct StepCtx {
  const Geo& g;
  const float* __restrict__ yv;
  const float* __restrict__ rk;
  float* __restrict__ out;       // UPD_NORMAL
  float* __restrict__ rho_next;  // UPD_FISTA
  float* __restrict__ y_next;
  float s, lam, alpha, tau, beta1;
  bool stencil;
  int aw;
  long long pl;
  __device__ StepCtx(const VolDesc& vd, const AdjOut& ao) : g(vd.g) {
    const int kk = vd.st->k;
    yv = (UPD == UPD_NORMAL) ? (ao.yin ? ao.yin : vd.rho[kk & 1]) : vd.y[kk & 1];
    rk = vd.rho[kk & 1];
    out = (UPD == UPD_NORMAL) ? (ao.out ? ao.out : vd.rho[(kk + 1) & 1]) : nullptr;
    rho_next = vd.rho[(kk + 1) & 1];
    y_next = vd.y[(kk + 1) & 1];
    s = (UPD == UPD_NORMAL) ? (float)vd.st->scale : 1.f;
    lam = vd.lam;
    alpha = vd.alpha;
    tau = (float)vd.st->tau;
    beta1 = (float)((double)kk / (kk + 3.0));      // (k+1-1)/(k+1+2)
    stencil = vd.reg_kind == 0;
    aw = vd.aw;
    pl = (long long)g.ny * g.nz;
  }
  __device__ __forceinline__ StencilVals load(long long i, float u) const {
    StencilVals v;
    v.c = yv[i];
    v.u = u;
    v.rk = (UPD == UPD_FISTA) ? rk[i] : 0.f;
    v.shell = false;
    if (stencil || alpha > 0.f) {
      const uint32_t r = g.f_nz.div((uint32_t)i);
      const int z = (int)((uint32_t)i - r * (uint32_t)g.nz);
      const int y = (int)g.f_ny.mod(r), x = (int)g.f_ny.div(r);
      // a 2D grid's projection axis (ny = 1) has no faces
      v.shell = x < aw || x >= g.nx - aw || (g.ny > 1 && (y < aw || y >= g.ny - aw)) || z < aw || z >= g.nz - aw;
      if (!stencil) return v;
      const long long row = i - z;
      // periodic neighbours (every axis is >= 4 long, so one wrap suffices, except the
      // projection axis of a 2D grid: length 1, every neighbour is the voxel itself and
      // its second differences vanish)
      auto wz = [&](int d) { int q = z + d; q += q < 0 ? g.nz : 0; q -= q >= g.nz ? g.nz : 0; return yv[row + q]; };
      auto wy = [&](int d) {
        if (g.ny == 1) return v.c;
        int q = y + d; q += q < 0 ? g.ny : 0; q -= q >= g.ny ? g.ny : 0;
        return yv[i + (long long)(q - y) * g.nz];
      };
      auto wx = [&](int d) {
        int q = x + d; q += q < 0 ? g.nx : 0; q -= q >= g.nx ? g.nx : 0;
        return yv[i + (long long)(q - x) * pl];
      };
      v.zm2 = wz(-2); v.zm1 = wz(-1); v.zp1 = wz(1); v.zp2 = wz(2);
      v.ym2 = wy(-2); v.ym1 = wy(-1); v.yp1 = wy(1); v.yp2 = wy(2);
      v.xm2 = wx(-2); v.xm1 = wx(-1); v.xp1 = wx(1); v.xp2 = wx(2);
    }
    return v;
  }
  // T^T T (s y) + alpha P_alpha^T P_alpha (s y).  No contraction into fused
  // multiply-adds here or in apply: the two kernels that inline these functions then
  // round every operation alike and finish a step bitwise identically.
  __device__ __forceinline__ float reg(const StencilVals& v) const {
#pragma clang fp contract(off)
    float t;
    if (!stencil) {
      t = s * v.c;
    } else {
      t = 18.f * (s * v.c);
      t += s * (v.zp2 + v.zm2) - 4.f * s * (v.zp1 + v.zm1);
      t += s * (v.yp2 + v.ym2) - 4.f * s * (v.yp1 + v.ym1);
      t += s * (v.xp2 + v.xm2) - 4.f * s * (v.xp1 + v.xm1);
    }
    if (alpha > 0.f && v.shell) t += alpha * (s * v.c);
    return t;
  }
  static constexpr int NV = UPD == UPD_NORMAL ? 2 : 3;
  // the update of voxel i and its terms of the FP64 sums
  __device__ __forceinline__ void apply(long long i, const StencilVals& v, double* acc) const {
#pragma clang fp contract(off)
    if constexpr (UPD == UPD_NORMAL) {
      const float o = v.u + lam * reg(v);
      out[i] = o;
      acc[0] += (double)(s * v.c) * (double)o;
      acc[1] += (double)o * (double)o;
    } else {
      const float yk = v.c;
      const float gr = v.u + lam * reg(v);
      const float rn = fmaxf(yk - tau * gr, 0.f);
      rho_next[i] = rn;
      y_next[i] = rn + beta1 * (rn - v.rk);
      const double dd = (double)rn - (double)yk;
      acc[0] += dd * dd;
      acc[1] += (double)rn * (double)rn;
      if (!isfinite(gr) || !isfinite(yk)) acc[2] += 1.0;   // max(NaN, 0) would hide it
    }
  }
};

// The block's FP64 sums into vd.partials[NV * lb ...] (k_vol_finish reduces them).
template <int NV>
__device__ __forceinline__ void store_step_partials(const VolDesc& vd, double* acc, double* red, int lb) {
  block_reduce_f64<NV>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) vd.partials[NV * lb + j] = acc[j];
  }
}

// Deterministic grid reduction: every block writes NV partials; the last block to
// arrive sums them in block order.  Returns true in thread 0 of the last block.
template <int NV>
__device__ __forceinline__ bool grid_reduce_last(double* v, double* partials, DevState* st, double* sh,
                                                 int blk, int nblk) {
  block_reduce_f64<NV>(v, sh);
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) partials[blk * NV + j] = v[j];
    __threadfence();
    const int prev = atomicAdd(&st->counter, 1);
    is_last = (prev == nblk - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  // the last block sums the partials: thread t takes blocks t, t + blockDim, ... in
  // order, then the fixed-order block reduction (the same result for any arrival order)
  __threadfence();
  double w[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) w[j] = 0.0;
  const volatile double* vp = partials;
  for (int bidx = threadIdx.x; bidx < nblk; bidx += blockDim.x) {
#pragma unroll
    for (int j = 0; j < NV; ++j) w[j] += vp[bidx * NV + j];
  }
  block_reduce_f64<NV>(w, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = w[j];
    st->counter = 0;
  }
  return threadIdx.x == 0;
}

// Adjoint pass 1: gather the class layout into a half plane, inverse y FFT, C2R
// along z, times the sensitivity:
//   OUT_SCALE_B      ao.out = b . v                          (A^T)
//   OUT_U            vd.u = b . v  (the A^T A part of a solver step; skipped once the
//                    volume's solve is done; k_vol_update finishes the step)
//   OUT_STEP_NORMAL  the step itself on the block's voxels with u = b . v (StepCtx),
//   OUT_STEP_FISTA   its FP64 sums in vd.partials[lb] for k_vol_finish (scalar model:
//                    one component)
// grid = ps * nx blocks (ps per x-plane); lb = the block's index among them.
template <int OUT>
__device__ __forceinline__ void plane_adj_body(const VolDesc& vd, int lb, const AdjOut& ao) {
  const Geo& g = vd.g;
  constexpr bool kStep = (OUT == OUT_STEP_NORMAL || OUT == OUT_STEP_FISTA);
  if constexpr (OUT == OUT_U || kStep) {
    if (vd.st->done) return;
  }
  extern __shared__ float2 lds[];
  const int pl = plane_lds(g);
  float2* twz = lds;
  float2* twy = twz + g.nz;
  float2* P0 = twy + g.ny;
  float2* P1 = P0 + pl;
  load_table(twz, vd.tw + vd.off[2], g.nz);
  load_table(twy, vd.tw + vd.off[1], g.ny);
  // ps workgroups per plane: all of them transform every column along y, workgroup h
  // then takes the z-transforms of the row pairs [j0, j1)
  const int h = lb / g.nx;
  const int x = plane_of_block(lb - h * g.nx, g.nx);
  const int j0 = h * g.npairs / g.ps, j1 = (h + 1) * g.npairs / g.ps;
  // vector model: out = sum_i b_i . v_i, the components added in order by the thread
  // that owns the voxel (a plane workgroup fills its CU, so components in workgroups of
  // their own would only queue behind each other)
  for (int comp = 0; comp < vd.ncomp; ++comp) {
  if (comp) __syncthreads();   // the previous component's store still reads the LDS planes
  const float2* src = vd.uperm + (long long)comp * g.hsz + (long long)x * g.plane;
  batched<8, float2>(g.plane, [&](int e) { return src[e]; }, [&](int e, float2 v) { P1[e] = v; });
  __syncthreads();
  for (int p = threadIdx.x; p < g.ny * g.nzh; p += blockDim.x) {
    const int qz = (int)g.f_ny.div((uint32_t)p), qy = p - qz * g.ny;
    bool cj;
    const int e = class_index_of(g, qy, qz, cj);
    const float2 v = P1[e];
    P0[qz * g.lsy + qy] = cj ? make_float2(v.x, -v.y) : v;
  }
  float2* X = fft_lines<+1>(P0, P1, twy, g.ny, g.nzh, g.lsy);
  float2* Z = c2r_rows_range(X, X == P0 ? P1 : P0, twz, g.ny, g.nz, j0, j1, plane_rowcols(g), g.f_nz);
  const int lsz = pad_odd(g.nz);
  const float* Xf = reinterpret_cast<const float*>(Z);
  // rows [2 j0, min(2 j1, ny)) of the plane; row y is in line (y >> 1) - j0
  const int y0 = 2 * j0, y1 = 2 * j1 < g.ny ? 2 * j1 : g.ny;
  auto vidx = [&](int p) {
    const int y = (int)g.f_nz.div((uint32_t)p), z = p - y * g.nz;
    return 2 * (((y >> 1) - j0) * lsz + z) + (y & 1);
  };
  const float* __restrict__ b = vd.b + (long long)comp * g.N;
  const long long pbase = (long long)x * g.ny * g.nz + (long long)y0 * g.nz;
  if constexpr (kStep) {
    // u = b . v of the block's voxels stays in registers: the step reads it there
    constexpr int UPD = OUT == OUT_STEP_NORMAL ? UPD_NORMAL : UPD_FISTA;
    constexpr int NV = StepCtx<UPD>::NV;
    __shared__ double red[64];
    const StepCtx<UPD> ctx(vd, ao);
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    const int n = (y1 - y0) * g.nz;
    // voxels whose loads are in flight together (half a 96 x 64 plane over 1024 threads
    // is one round; 3 measured 1.7 % faster per update than 2 at 96 x 96 x 64)
    constexpr int U = 3;
    for (int p = threadIdx.x; p < n; p += U * (int)blockDim.x) {
      StencilVals v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int pq = p + q * (int)blockDim.x;
        // a rounded product, as the stored u that k_vol_update reads (no contraction
        // into the step's sums), so both ways of finishing a step agree bitwise
        if (pq < n) v[q] = ctx.load(pbase + pq, __fmul_rn(b[pbase + pq], Xf[vidx(pq + y0 * g.nz)]));
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int pq = p + q * (int)blockDim.x;
        if (pq < n) ctx.apply(pbase + pq, v[q], acc);
      }
    }
    store_step_partials<NV>(vd, acc, red, lb);
    return;
  }
  float* __restrict__ out = (OUT == OUT_U) ? vd.u : ao.out;
  if (comp == 0) {
    batched<8, float>((y1 - y0) * g.nz, [&](int p) { return b[pbase + p]; },
                      [&](int p, float bv) { out[pbase + p] = bv * Xf[vidx(p + y0 * g.nz)]; });
  } else {
    batched<8, float>((y1 - y0) * g.nz, [&](int p) { return b[pbase + p]; },
                      [&](int p, float bv) { out[pbase + p] += bv * Xf[vidx(p + y0 * g.nz)]; });
  }
  }
}
template <int OUT>
__global__ __launch_bounds__(1024) void k_plane_adj(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                    AdjOut ao) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  plane_adj_body<OUT>(vd, lb, ao);
}

// A solver update's adjoint plane pass and step (OUT_STEP_FISTA), then, in the same
// workgroup, the next update's forward plane pass on the y^{k+1} the step just wrote
// (u = b . y^{k+1}, as k_plane_fwd<SRC_FISTA_Y> forms it): a plane's forward pass needs
// only that plane's y, so with one workgroup per x-plane (ps = 1) no other block is
// awaited, and the next update starts at its class pass.  If this step ends the solve,
// the extra forward pass is unused.  grid = nx blocks (ps must be 1).
__global__ __launch_bounds__(1024) void k_step_and_fwd(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                       AdjOut ao) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  if (vd.st->done) return;
  const float* ynext = vd.y[(vd.st->k + 1) & 1];
  plane_adj_body<OUT_STEP_FISTA>(vd, lb, ao);
  __syncthreads();   // the block's stores of y^{k+1} are visible to it; the LDS is free
  plane_fwd_body<SRC_PLAIN>(vd, lb, ynext);
}

// The two passes after the fused class pass in A then A^T, in one launch: both read only
// what that pass wrote, so blocks [0, ps nx) run the adjoint plane pass (ao.out = b . v)
// while the others run the small-grid inverse pass that writes the portraits d.  The
// plane blocks come first (their XCD-aware plane order assumes block ids 0 .. ps nx - 1);
// the small-grid blocks run beside them.  Both bodies loop over blockDim (512 or 1024).
__global__ __launch_bounds__(1024) void k_adj_and_store(const VolDesc* __restrict__ vds, AdjOut ao, float* __restrict__ d) {
  const VolDesc& vd = vds[0];
  const int nplane = vd.g.ps * vd.g.nx;
  if ((int)blockIdx.x < nplane) plane_adj_body<OUT_SCALE_B>(vd, blockIdx.x, ao);
  else small_inv_body<EPI_STORE>(vd, blockIdx.x - nplane, d);
}

// Blocks of the volume-wide update pass, each a contiguous run of whole UPD_THREADS-voxel
// tiles: about 2048 voxels per block, at most 256 blocks per volume (their FP64
// partials are summed by k_vol_finish).  512 threads let two blocks share a CU, which
// matters when a batch launches thousands of them.
constexpr int UPD_THREADS = 512;
__host__ __device__ inline int update_blocks(long long n) {
  long long b = (n + 2047) / 2048;
  return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}

// Finishes a solver step after k_plane_adj<OUT_U> left u = b . v (see StepCtx).  Each
// block leaves its FP64 sums in vd.partials; k_vol_finish reduces them and updates the
// state.  grid = vd.nb_upd blocks of UPD_THREADS threads per volume.
template <int UPD>
__global__ __launch_bounds__(UPD_THREADS) void k_vol_update(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks,
                                                    AdjOut ao) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  const Geo& g = vd.g;
  if (vd.st->done) return;
  __shared__ double red[64];
  const StepCtx<UPD> ctx(vd, ao);
  const float* __restrict__ u = vd.u;
  const long long N = g.N;
  const int nb = vd.nb_upd;
  constexpr int T = UPD_THREADS;
  const long long chunk = ((N + nb - 1) / nb + T - 1) / T * T;
  // XCD-aware: blocks of one XCD take consecutive chunks (the planes k_plane_adj
  // wrote on that XCD, and their x-neighbours)
  const long long i0 = (long long)plane_of_block(lb, nb) * chunk;
  const long long i1 = i0 + chunk < N ? i0 + chunk : N;
  constexpr int U = 4;
  constexpr int NV = StepCtx<UPD>::NV;
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  for (long long i = i0 + threadIdx.x; i < i1; i += U * T) {
    StencilVals v[U];
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (i + q * T < i1) v[q] = ctx.load(i + q * T, u[i + q * T]);
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (i + q * T >= i1) break;
      ctx.apply(i + q * T, v[q], acc);
    }
  }
  store_step_partials<NV>(vd, acc, red, lb);
}

// Sums the block partials of k_vol_update in a fixed order (thread t takes blocks
// t, t + 256, ..., then the fixed-order block reduction) and advances the state.
// One block per volume; the kernel boundary orders it after every partial store.
template <int UPD>
__global__ __launch_bounds__(256) void k_vol_finish(const VolDesc* __restrict__ vds, const int2* __restrict__ tasks) {
  int lb;
  const VolDesc& vd = vol_of(vds, tasks, lb);
  DevState* st = vd.st;
  if (st->done) return;
  __shared__ double red[64];
  constexpr int NV = UPD == UPD_NORMAL ? 2 : 3;
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  for (int b = threadIdx.x; b < vd.nb_upd; b += blockDim.x) {
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] += vd.partials[b * NV + j];
  }
  block_reduce_f64<NV>(acc, red);
  if (threadIdx.x != 0) return;
  const int kk = st->k;
  if constexpr (UPD == UPD_NORMAL) {
    st->lmax = acc[0];
    st->scale = 1.0 / sqrt(acc[1]);
    if (!(acc[0] == acc[0]) || !(acc[1] < 1e300)) st->nonfinite = 1.0;
    st->k = kk + 1;
    if (kk >= st->kmax) st->done = 1;
  } else {
    double r;
    if (acc[1] == 0.0) r = (acc[0] == 0.0) ? 0.0 : __builtin_inf();
    else r = sqrt(acc[0]) / sqrt(acc[1]);
    st->rel_step = r;
    st->last_k = kk;
    const int hi = kk - vd.k_first;
    if (vd.hist && hi >= 0 && hi < vd.hist_len) vd.hist[hi] = r;
    if (acc[2] != 0.0 || !(acc[0] == acc[0]) || !(acc[1] == acc[1]) || acc[1] > 1e300) {
      st->nonfinite = 1.0;
      st->done = 1;
    }
    // tol = 0 never stops early (not even at r_k = 0): the run takes max_iter updates
    if ((st->tol > 0.0 && r <= st->tol) || kk >= st->kmax) st->done = 1;
    st->k = kk + 1;
  }
}

// ============================================================================ MHAD
// Multi-harmonic anti-differentiation (App. D, eq. mhadM): the native image on the
// portrait grid from the portraits, per line along the drive axis (x'):
//   rho_N^(q) = sum_k c_k^{-1} conj(f^(q))^{k-1} d_k^(q) / (sum_k |f^(q)|^{2(k-1)} + lambda),
// f^(q) = 2i sin(2 pi q / m) (the central difference u[j+1] - u[j-1]).  A block takes
// CB lines (consecutive (y', z') columns, so the loads and stores are coalesced), FFTs
// each harmonic's lines in LDS and accumulates the weighted spectra, then divides and
// transforms back.  grid = ceil(C / CB), C = my' mz'; dynamic LDS (m + 3 CB ls) float2
// + m floats, ls = pad_odd(m).
struct MhadW {
  int ord[32];        // k - 1 per harmonic
  double cinv[32];    // 1 / c_k
};

__global__ __launch_bounds__(256) void k_mhad(const float* __restrict__ d, int K, MhadW wk, double lam, int m,
                                              long long C, int CB, float* __restrict__ out) {
  extern __shared__ float2 sm[];
  const int ls = pad_odd(m);
  float2* tw = sm;
  float2* A0 = tw + m;
  float2* A1 = A0 + CB * ls;
  float2* acc = A1 + CB * ls;
  float* den = reinterpret_cast<float*>(acc + CB * ls);
  const long long c0 = (long long)blockIdx.x * CB;
  const int nc = (int)(C - c0 < CB ? C - c0 : CB);
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)t / (double)m, &sn, &cs);
    tw[t] = make_float2((float)cs, (float)-sn);
    double sum = lam;
    for (int i = 0; i < K; ++i) sum += pow(4.0 * sn * sn, (double)wk.ord[i]);
    den[t] = (float)sum;
  }
  for (int p = threadIdx.x; p < CB * ls; p += blockDim.x) acc[p] = make_float2(0.f, 0.f);
  for (int i = 0; i < K; ++i) {
    __syncthreads();
    for (int p = threadIdx.x; p < m * nc; p += blockDim.x) {
      const int x = p / nc, c = p - x * nc;
      A0[c * ls + x] = make_float2(d[(long long)i * m * C + (long long)x * C + c0 + c], 0.f);
    }
    const float2* F = fft_lines<-1>(A0, A1, tw, m, nc, ls);
    const int n = wk.ord[i];
    for (int p = threadIdx.x; p < m * nc; p += blockDim.x) {
      const int c = p / m, q = p - c * m;
      // c_k^{-1} (-2i sin)^n = c_k^{-1} (2 sin)^n (-i)^n
      const double mag = wk.cinv[i] * pow(2.0 * sinpi(2.0 * (double)q / (double)m), (double)n);
      float2 w;
      switch (n & 3) {
        case 0: w = make_float2((float)mag, 0.f); break;
        case 1: w = make_float2(0.f, (float)-mag); break;
        case 2: w = make_float2((float)-mag, 0.f); break;
        default: w = make_float2(0.f, (float)mag); break;
      }
      const float2 v = F[c * ls + q];
      float2& a = acc[c * ls + q];
      a.x += w.x * v.x - w.y * v.y;
      a.y += w.x * v.y + w.y * v.x;
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < m * nc; p += blockDim.x) {
    const int c = p / m, q = p - c * m;
    const float inv = 1.f / den[q];
    A0[c * ls + q] = make_float2(acc[c * ls + q].x * inv, acc[c * ls + q].y * inv);
  }
  const float2* G = fft_lines<+1>(A0, A1, tw, m, nc, ls);
  const float invm = 1.f / (float)m;
  for (int p = threadIdx.x; p < m * nc; p += blockDim.x) {
    const int x = p / nc, c = p - x * nc;
    out[(long long)x * C + c0 + c] = G[c * ls + x].x * invm;
  }
}

// y^{k0} = rho^{k0} + (k0-1)/(k0+2) (rho^{k0} - rho^{k0-1}) for a (re)started solve.
// y^{k0} = rho^{k0} + beta (rho^{k0} - rho^{k0-1}), rounded as the step forms y^{k+1}
// (no contraction), so a resumed solve continues bitwise as the uninterrupted one.
__global__ void k_fista_init(long long n, const float* __restrict__ rk, const float* __restrict__ rkm1,
                             float beta, float* __restrict__ y) {
#pragma clang fp contract(off)
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float r = rk[i];
    y[i] = r + beta * (r - rkm1[i]);
  }
}

// ============================================================================ plan-time kernels
// Twiddle tables exp(-2 pi i t / n), FP64 evaluation, FP32 and FP64 copies.
__global__ void k_twiddles(int n, float2* __restrict__ t32, double2* __restrict__ t64) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)t / (double)n, &s, &c);
    if (t32) t32[t] = make_float2((float)c, (float)-s);
    if (t64) t64[t] = make_double2(c, -s);
  }
}

// Gaussian sensitivity, peak 1 at the geometric centre ((N-1)/2 voxel).
__global__ void k_sensitivity(Geo g, double vox, double sx, double sy, double sz, float* __restrict__ b) {
  const long long n = g.N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(i % g.nz);
    const int y = (int)((i / g.nz) % g.ny);
    const int x = (int)(i / ((long long)g.ny * g.nz));
    const double ax = (x - 0.5 * (g.nx - 1)) * vox / sx;
    const double ay = (y - 0.5 * (g.ny - 1)) * vox / sy;
    const double az = (z - 0.5 * (g.nz - 1)) * vox / sz;
    b[i] = (float)exp(-0.5 * (ax * ax + ay * ay + az * az));
  }
}

__device__ __forceinline__ int signed_offset(int i, int n) { return (2 * i < n) ? i : i - n; }

// Drive-axis profiles f_k(x) = L^(order_k)(a vox w(x)) (symmetric mean at x = nx/2
// for even nx), their FFT along x in FP64, and ||f_k||^2.  grid = K blocks.
__global__ __launch_bounds__(256) void k_psf_profile(int nx, const int* __restrict__ order, double a_vox,
                                                     const double2* __restrict__ tw64,
                                                     double* __restrict__ prof, double2* __restrict__ fhat,
                                                     double* __restrict__ fnorm2) {
  extern __shared__ double2 lds64[];
  double2* tw = lds64;
  double2* X = tw + nx;
  double2* X1 = X + nx;
  __shared__ double red[64];
  const int k = blockIdx.x;
  const int n = order[k];
  load_table(tw, tw64, nx);
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    double f;
    if ((nx % 2 == 0) && 2 * i == nx) {
      const double u = a_vox * (nx / 2);
      f = 0.5 * (langevin_deriv_dev(n, u) + langevin_deriv_dev(n, -u));
    } else {
      f = langevin_deriv_dev(n, a_vox * signed_offset(i, nx));
    }
    prof[(long long)k * nx + i] = f;
    X[i] = make_double2(f, 0.0);
    acc[0] += f * f;
  }
  const double2* F = fft_lines<-1>(X, X1, tw, nx, 1, nx);
  for (int i = threadIdx.x; i < nx; i += blockDim.x) fhat[(long long)k * nx + i] = F[i];
  block_reduce_f64<1>(acc, red);
  if (threadIdx.x == 0) fnorm2[k] = acc[0];
}

// Transverse envelope E(y, z) = L'(a r)/r, E(0) = L'(0) 4 asinh(1)/vox, one row per
// block, then FFT along z (FP64).  Also per-row sum of E^2.  grid = ny blocks.
__global__ __launch_bounds__(256) void k_psf_env_rows(int ny, int nz, double a, double vox,
                                                      const double2* __restrict__ tw64z,
                                                      double* __restrict__ env, double2* __restrict__ tmp,
                                                      double* __restrict__ rowsum) {
  extern __shared__ double2 lds64[];
  double2* tw = lds64;
  double2* X = tw + nz;
  double2* X1 = X + nz;
  __shared__ double red[64];
  const int y = blockIdx.x;
  load_table(tw, tw64z, nz);
  double acc[1] = {0.0};
  const double wy = signed_offset(y, ny) * vox;
  for (int z = threadIdx.x; z < nz; z += blockDim.x) {
    const double wz = signed_offset(z, nz) * vox;
    const double r = sqrt(wy * wy + wz * wz);
    double e;
    if (r > 0.0) e = langevin_deriv_dev(1, a * r) / r;
    else e = (1.0 / 3.0) * 4.0 * asinh(1.0) / vox;
    env[(long long)y * nz + z] = e;
    X[z] = make_double2(e, 0.0);
    acc[0] += e * e;
  }
  const double2* F = fft_lines<-1>(X, X1, tw, nz, 1, nz);
  for (int z = threadIdx.x; z < nz; z += blockDim.x) tmp[(long long)y * nz + z] = F[z];
  block_reduce_f64<1>(acc, red);
  if (threadIdx.x == 0) rowsum[y] = acc[0];
}

// FFT along y of the row-transformed envelope, one column per block (qz <= nz/2).
__global__ __launch_bounds__(256) void k_psf_env_cols(int ny, int nz, const double2* __restrict__ tw64y,
                                                      const double2* __restrict__ tmp, double2* __restrict__ ehat) {
  extern __shared__ double2 lds64[];
  double2* tw = lds64;
  double2* X = tw + ny;
  double2* X1 = X + ny;
  const int qz = blockIdx.x;
  load_table(tw, tw64y, ny);
  for (int y = threadIdx.x; y < ny; y += blockDim.x) X[y] = tmp[(long long)y * nz + qz];
  const double2* F = fft_lines<-1>(X, X1, tw, ny, 1, ny);
  for (int y = threadIdx.x; y < ny; y += blockDim.x) ehat[(long long)y * (nz / 2 + 1) + qz] = F[y];
}

// scale[k] = 1 / (||f_k|| ||E|| N)   (unit-norm PSF, unnormalised FFTs downstream)
__global__ void k_psf_scales(int K, int ny, long long N, const double* __restrict__ fnorm2,
                             const double* __restrict__ rowsum, double* __restrict__ scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double e2 = 0.0;
    for (int y = 0; y < ny; ++y) e2 += rowsum[y];
    for (int k = 0; k < K; ++k) scale[k] = 1.0 / (sqrt(fnorm2[k]) * sqrt(e2) * (double)N);
  }
}

// Spectrum in the class layout [k][class][q'x][jx][member], scaled by 1/N:
// Hs = F_k(qx) Ehat(qy, qz) scale_k.  Compact form stores Re (odd order) or Im
// (even order); complex form stores both.
__global__ void k_psf_assemble(Geo g, const double2* __restrict__ fhat, const double2* __restrict__ ehat,
                               const double* __restrict__ scale, uint32_t imag_mask, int compact,
                               void* __restrict__ hs) {
  const long long total = (long long)g.K * g.hsz;
  const int per_cls = g.mx * g.S;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t / g.hsz);
    const long long r = t % g.hsz;
    const int c = (int)(r / per_cls);
    const int r2 = (int)(r % per_cls);
    const int qxp = r2 / g.S, w = r2 % g.S;
    const int jx = w / g.nmem, m = w % g.nmem;
    const int qx = qxp + jx * g.mx;
    const int qy = (c / g.mzh) + (m / g.sz) * g.my;
    const int qz = (c % g.mzh) + (m % g.sz) * g.mz;
    double2 e;
    if (2 * qz <= g.nz) e = ehat[(long long)qy * g.nzh + qz];
    else { e = ehat[(long long)((g.ny - qy) % g.ny) * g.nzh + (g.nz - qz)]; e.y = -e.y; }
    const double2 f = fhat[(long long)k * g.nx + qx];
    const double s = scale[k];
    const double hr = (f.x * e.x - f.y * e.y) * s;
    const double hi = (f.x * e.y + f.y * e.x) * s;
    if (compact) reinterpret_cast<float*>(hs)[t] = (float)(((imag_mask >> k) & 1u) ? hi : hr);
    else reinterpret_cast<float2*>(hs)[t] = make_float2((float)hr, (float)hi);
  }
}

// User PSF spectra: FFT along x of the class-layout yz spectrum of h_k, scaled by
// 1/N, stored complex in the class layout.  grid = ncls/cpw blocks, cpw*nmem lines.
__global__ __launch_bounds__(1024) void k_class_hcopy(Geo g, int k, const float2* __restrict__ uperm,
                                                      float2* __restrict__ hs, const float2* __restrict__ tw_x) {
  extern __shared__ float2 lds[];
  float2* twx = lds;
  const int W = g.cpw * g.nmem;
  float2* U0 = twx + g.nx;
  float2* U1 = U0 + W * g.lsx;
  load_table(twx, tw_x, g.nx);
  const int c0 = blockIdx.x * g.cpw;
  batched<8, float2>(g.nx * W,
                     [&](int p) {
                       const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
                       return uperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e];
                     },
                     [&](int p, float2 v) {
                       const int xx = (int)g.f_W.div((uint32_t)p), e = p - xx * W;
                       U0[e * g.lsx + xx] = v;
                     });
  const float2* Ul = fft_lines<-1>(U0, U1, twx, g.nx, W, g.lsx);
  const float invN = (float)(1.0 / (double)g.N);
  const int per_cls = g.mx * g.S;
  for (int t = threadIdx.x; t < g.cpw * per_cls; t += blockDim.x) {
    const int cl = (int)g.f_mxS.div((uint32_t)t), r2 = t - cl * per_cls;
    const int qxp = (int)g.f_S.div((uint32_t)r2), w = r2 - qxp * g.S;
    const int jx = (int)g.f_nmem.div((uint32_t)w), m = w - jx * g.nmem;
    const float2 v = Ul[(cl * g.nmem + m) * g.lsx + qxp + jx * g.mx];
    hs[(long long)k * g.hsz + (long long)c0 * per_cls + t] = make_float2(v.x * invN, v.y * invN);
  }
}

// Flags of the PSF blocks that are not identically zero: blockIdx.x = j selects the
// (component, harmonic) block psf + j * N, blockIdx.y = s one of gridDim.y strided
// shares of it; flags[j * gridDim.y + s] = any nonzero in the share.
__global__ __launch_bounds__(256) void k_nonzero_blocks(const float* __restrict__ psf, long long N,
                                                        int* __restrict__ flags) {
  const float* p = psf + (long long)blockIdx.x * N;
  const long long step = (long long)gridDim.y * blockDim.x;
  int any = 0;
  for (long long i = (long long)blockIdx.y * blockDim.x + threadIdx.x; i < N; i += step) any |= (p[i] != 0.f);
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[blockIdx.x * gridDim.y + blockIdx.y] = any;
}

// Back from the class layout to [k][nx][ny][nzh] complex, times N (tests/tools).
__global__ void k_spectrum_export(Geo g, const void* __restrict__ hs, uint32_t imag_mask, int compact,
                                  float2* __restrict__ out) {
  const long long per_k = (long long)g.nx * g.ny * g.nzh;
  const long long total = (long long)g.K * per_k;
  const int per_cls = g.mx * g.S;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(t / per_k);
    long long r = t % per_k;
    const int qz = (int)(r % g.nzh);
    const int qy = (int)((r / g.nzh) % g.ny);
    const int qx = (int)(r / ((long long)g.nzh * g.ny));
    bool cj;
    const int e = class_index_of(g, qy, qz, cj);  // member index in the plane layout
    const int c = e / g.nmem, m = e % g.nmem;
    const int qxs = cj ? (g.nx - qx) % g.nx : qx;   // conjugate partner also negates qx
    const int qxp = qxs % g.mx, jx = qxs / g.mx;
    const long long idx = (long long)k * g.hsz + (long long)c * per_cls + qxp * g.S + jx * g.nmem + m;
    float2 v;
    if (compact) {
      const float f = reinterpret_cast<const float*>(hs)[idx];
      v = ((imag_mask >> k) & 1u) ? make_float2(0.f, f) : make_float2(f, 0.f);
    } else v = reinterpret_cast<const float2*>(hs)[idx];
    if (cj) v.y = -v.y;
    const float Nf = (float)g.N;
    out[t] = make_float2(v.x * Nf, v.y * Nf);
  }
}

// ============================================================================ small helpers
// Philox4x32-10 (Salmon et al., SC'11) uniform (w + 0.5)/2^32 start vector, and
// FP64 partials of its squared norm; last block stores 1/||x0|| in st->scale.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__global__ void k_philox_uniform(long long n, uint64_t seed, uint32_t stream, float* __restrict__ out,
                                 double* __restrict__ partials, DevState* st) {
  __shared__ double red[64];
  double acc[1] = {0.0};
  const long long nblk = (n + 3) / 4;
  for (long long bi = blockIdx.x * (long long)blockDim.x + threadIdx.x; bi < nblk; bi += (long long)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)bi, stream, 0u, 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    for (int j = 0; j < 4; ++j) {
      const long long i = bi * 4 + j;
      if (i < n) {
        const double u = ((double)c[j] + 0.5) / 4294967296.0;
        out[i] = (float)u;
        acc[0] += (double)(float)u * (double)(float)u;
      }
    }
  }
  if (grid_reduce_last<1>(acc, partials, st, red, blockIdx.x, gridDim.x)) st->scale = 1.0 / sqrt(acc[0]);
}

// Raw Philox words for the known-answer test.
__global__ void k_philox_words(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                               uint32_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    uint32_t c[4] = {c0, c1, c2, c3};
    philox4x32_10(c, k0, k1);
    for (int j = 0; j < 4; ++j) out[j] = c[j];
  }
}

}  // namespace mh3d
