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
  const int qzr = qz % g.mz;
  int yy = qy, zz = qz;
  cj = false;
  if (2 * qzr > g.mz) {            // stored as the conjugate of (ny - qy, nz - qz)
    yy = (g.ny - qy) % g.ny;
    zz = g.nz - qz;
    cj = true;
  }
  const int c = (yy % g.my) * g.mzh + (zz % g.mz);
  const int m = (yy / g.my) * g.sz + (zz / g.mz);
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

// Complex elements of one LDS plane buffer (x-plane kernels) / small-grid buffer.
__host__ __device__ inline int plane_lds(const Geo& g) {
  const int a = g.npairs * g.nz, b = g.ny * g.nzh;
  return a > b ? a : b;
}
__host__ __device__ inline int small_lds(const Geo& g) {
  const int a = g.spairs * g.mz, b = g.xb * g.my * g.mzh;
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

// ============================================================================ pass 1: x-plane R2C
enum { SRC_PLAIN = 0, SRC_RAW = 1, SRC_FISTA_Y = 2, SRC_SCALED = 3 };

// Value fed to the forward FFT at flat voxel i.
template <int SRC>
__device__ __forceinline__ float plane_source(long long i, const float* __restrict__ a,
                                              const float* __restrict__ a2,
                                              const float* __restrict__ b, float coef) {
  if constexpr (SRC == SRC_PLAIN) return b[i] * a[i];
  else if constexpr (SRC == SRC_RAW) return a[i];
  else if constexpr (SRC == SRC_FISTA_Y) {     // y = rho^k + beta (rho^k - rho^{k-1})
    float r = a[i];
    return b[i] * (r + coef * (r - a2[i]));
  } else return b[i] * (coef * a[i]);          // SRC_SCALED
}

// R2C along z of nrows real rows held as packed pairs Z[j][nz] in *a (row 2j in .x,
// row 2j+1 in .y): FFT each pair, then split into half spectra X[row][0..nz/2]
// (row stride row_stride_out).  Returns the buffer holding X (a or b).
__device__ float2* r2c_rows(float2* a, float2* b, const float2* twz, int nrows, int nz, int nzh,
                            int row_stride_out, int npairs) {
  float2* Z = fft_lds<-1>(a, b, twz, nz, npairs, LineMap{npairs, 0, nz, 1}, false);
  float2* X = (Z == a) ? b : a;
  const int items = npairs * nzh;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int j = it / nzh, q = it % nzh;
    const float2 zq = Z[j * nz + q];
    const float2 zm = Z[j * nz + (nz - q) % nz];
    // A = (Z(q) + conj Z(-q))/2 ; B = (Z(q) - conj Z(-q))/(2i)
    X[(2 * j) * row_stride_out + q] = make_float2(0.5f * (zq.x + zm.x), 0.5f * (zq.y - zm.y));
    if (2 * j + 1 < nrows)
      X[(2 * j + 1) * row_stride_out + q] = make_float2(0.5f * (zq.y + zm.y), -0.5f * (zq.x - zm.x));
  }
  __syncthreads();
  return X;
}

// C2R along z: half spectra X[row][nzh] (row stride row_stride_in) in *a -> packed
// pairs Z[j][nz] (Z = A + iB with Hermitian extension), inverse FFT.  The
// imaginary parts of the q = 0 and q = nz/2 bins are dropped (they vanish for a
// Hermitian input).  Returns the buffer holding the packed real rows.
__device__ float2* c2r_rows(float2* a, float2* b, const float2* twz, int nrows, int nz, int nzh,
                            int row_stride_in, int npairs) {
  const int items = npairs * nz;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int j = it / nz, q = it % nz;
    const bool up = 2 * q > nz;
    const int qq = up ? nz - q : q;
    float2 x = a[(2 * j) * row_stride_in + qq];
    float2 y = (2 * j + 1 < nrows) ? a[(2 * j + 1) * row_stride_in + qq] : make_float2(0.f, 0.f);
    if (qq == 0 || 2 * qq == nz) { x.y = 0.f; y.y = 0.f; }
    if (up) { x.y = -x.y; y.y = -y.y; }
    b[it] = make_float2(x.x - y.y, x.y + y.x);      // x + i y
  }
  return fft_lds<+1>(b, a, twz, nz, npairs, LineMap{npairs, 0, nz, 1}, false);
}

// Forward pass 1.  grid = nx blocks (block -> plane).
// LDS: tables (nz + ny) + two plane buffers of max(npairs*nz, ny*nzh) complex.
template <int SRC>
__global__ __launch_bounds__(1024) void k_plane_fwd(Geo g, const float* __restrict__ a,
                                                    const float* __restrict__ a2,
                                                    const float* __restrict__ b, float coef,
                                                    const DevState* __restrict__ st,
                                                    float2* __restrict__ uperm,
                                                    const float2* __restrict__ tw_y,
                                                    const float2* __restrict__ tw_z) {
  if constexpr (SRC == SRC_FISTA_Y || SRC == SRC_SCALED) {
    if (st->done) return;
  }
  extern __shared__ float2 lds[];
  const int pl = plane_lds(g);
  float2* twz = lds;
  float2* twy = twz + g.nz;
  float2* P0 = twy + g.ny;
  float2* P1 = P0 + pl;
  const int x = blockIdx.x;
  load_table(twz, tw_z, g.nz);
  load_table(twy, tw_y, g.ny);
  float c = coef;
  if constexpr (SRC == SRC_FISTA_Y) c = (float)((st->k - 1.0) / (st->k + 2.0));
  if constexpr (SRC == SRC_SCALED) c = (float)st->scale;
  const long long pbase = (long long)x * g.ny * g.nz;
  const int nyz = g.ny * g.nz;
  float* Zf = reinterpret_cast<float*>(P0);
  for (int p = threadIdx.x; p < nyz; p += blockDim.x) {
    const int y = p / g.nz, z = p % g.nz;
    Zf[2 * ((y >> 1) * g.nz + z) + (y & 1)] = plane_source<SRC>(pbase + p, a, a2, b, c);
  }
  if (g.ny & 1) {
    for (int z = threadIdx.x; z < g.nz; z += blockDim.x) Zf[2 * ((g.ny >> 1) * g.nz + z) + 1] = 0.f;
  }
  float2* X = r2c_rows(P0, P1, twz, g.ny, g.nz, g.nzh, g.nzh, g.npairs);
  float2* Y = fft_lds<-1>(X, X == P0 ? P1 : P0, twy, g.ny, g.nzh, LineMap{g.nzh, 0, 1, g.nzh}, true);
  float2* dst = uperm + (long long)x * g.plane;
  for (int e = threadIdx.x; e < g.plane; e += blockDim.x) {
    bool cj;
    const int src = halfplane_of_member(g, e, cj);
    const float2 v = Y[src];
    dst[e] = cj ? make_float2(v.x, -v.y) : v;
  }
}

// ============================================================================ pass 2: classes
// HC = 0: compact spectra (one float per element; harmonic k is real if bit k of
// imag_mask is clear, purely imaginary if set).  HC = 1: complex spectra.
template <int HC, int E>
struct HLoad {
  float2 v[E];
  __device__ __forceinline__ void load(const void* base, long long off) {
    if constexpr (HC == 0) {
      const float* p = reinterpret_cast<const float*>(base) + off;
      if constexpr (E % 4 == 0) {
#pragma unroll
        for (int i = 0; i < E; i += 4) {
          float4 t = *reinterpret_cast<const float4*>(p + i);
          v[i] = make_float2(t.x, 0.f); v[i + 1] = make_float2(t.y, 0.f);
          v[i + 2] = make_float2(t.z, 0.f); v[i + 3] = make_float2(t.w, 0.f);
        }
      } else if constexpr (E % 2 == 0) {
#pragma unroll
        for (int i = 0; i < E; i += 2) {
          float2 t = *reinterpret_cast<const float2*>(p + i);
          v[i] = make_float2(t.x, 0.f); v[i + 1] = make_float2(t.y, 0.f);
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = make_float2(p[i], 0.f);
      }
    } else {
      const float2* p = reinterpret_cast<const float2*>(base) + off;
      if constexpr (E % 2 == 0) {
#pragma unroll
        for (int i = 0; i < E; i += 2) {
          float4 t = *reinterpret_cast<const float4*>(p + i);
          v[i] = make_float2(t.x, t.y); v[i + 1] = make_float2(t.z, t.w);
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = p[i];
      }
    }
  }
};

// LDS layout of the class kernels: tables (nx + mx), U0/U1 (nx*W each), F0/F1
// (K*cpw*mx each), W = cpw*nmem.
__host__ __device__ inline size_t class_lds_elems(const Geo& g) {
  const size_t W = (size_t)g.cpw * g.nmem;
  return (size_t)g.nx + g.mx + 2 * (size_t)g.nx * W + 2 * (size_t)g.K * g.cpw * g.mx;
}

// Forward pass 2.  grid = ncls/cpw blocks of cpw*mx*S/E threads.
template <int HC, int E>
__global__ __launch_bounds__(1024) void k_class_fwd(Geo g, const float2* __restrict__ uperm,
                                                    const void* __restrict__ hs, uint32_t imag_mask,
                                                    const DevState* __restrict__ st,
                                                    float2* __restrict__ G,
                                                    const float2* __restrict__ tw_x,
                                                    const float2* __restrict__ tw_mx) {
  if (st && st->done) return;
  extern __shared__ float2 lds[];
  const int W = g.cpw * g.nmem;
  float2* twx = lds;
  float2* twm = twx + g.nx;
  float2* U0 = twm + g.mx;
  float2* U1 = U0 + g.nx * W;
  float2* F0 = U1 + g.nx * W;
  float2* F1 = F0 + g.K * g.cpw * g.mx;
  load_table(twx, tw_x, g.nx);
  load_table(twm, tw_mx, g.mx);
  const int c0 = blockIdx.x * g.cpw;
  for (int p = threadIdx.x; p < g.nx * W; p += blockDim.x) {
    const int xx = p / W, e = p % W;
    U0[p] = uperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e];
  }
  const float2* U = fft_lds<-1>(U0, U1, twx, g.nx, W, LineMap{W, 0, 1, W}, true);
  // this thread's E spectrum elements: all share class cl and folded frequency qxp
  const int e0 = threadIdx.x * E;
  const int per_cls = g.mx * g.S;
  const int cl = e0 / per_cls;
  const int rem = e0 % per_cls;
  const int qxp = rem / g.S;
  const int within = rem % g.S;
  float2 ur[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int w = within + i;
    const int jx = w / g.nmem, m = w % g.nmem;
    ur[i] = U[(qxp + jx * g.mx) * W + cl * g.nmem + m];
  }
  const int LG = g.S / E;
  const long long hoff0 = (long long)c0 * per_cls + e0;
  HLoad<HC, E> hc, hn;
  hc.load(hs, hoff0);
  for (int k = 0; k < g.K; ++k) {
    if (k + 1 < g.K) hn.load(hs, (long long)(k + 1) * g.hsz + hoff0);
    float2 acc = make_float2(0.f, 0.f);
    if constexpr (HC == 0) {
#pragma unroll
      for (int i = 0; i < E; ++i) { acc.x += hc.v[i].x * ur[i].x; acc.y += hc.v[i].x * ur[i].y; }
      if ((imag_mask >> k) & 1u) acc = make_float2(-acc.y, acc.x);
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) acc = cadd(acc, cmul(hc.v[i], ur[i]));
    }
    for (int o = LG >> 1; o >= 1; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
    }
    if ((threadIdx.x % LG) == 0) F0[(k * g.cpw + cl) * g.mx + qxp] = acc;
    hc = hn;
  }
  const float2* F = fft_lds<+1>(F0, F1, twm, g.mx, g.K * g.cpw, LineMap{g.K * g.cpw, 0, g.mx, 1}, false);
  const int nxb = g.mx / g.xb;
  const int per_k = g.cpw * g.mx;
  for (int p = threadIdx.x; p < g.K * per_k; p += blockDim.x) {
    const int k = p / per_k, r = p % per_k;
    const int xbi = r / (g.cpw * g.xb), r2 = r % (g.cpw * g.xb);
    const int c = r2 / g.xb, xi = r2 % g.xb;
    G[(((long long)k * nxb + xbi) * g.ncls + c0 + c) * g.xb + xi] = F[(k * g.cpw + c) * g.mx + xbi * g.xb + xi];
  }
}

// Adjoint pass 2.  Same grid and LDS as k_class_fwd.
template <int HC, int E>
__global__ __launch_bounds__(1024) void k_class_adj(Geo g, const float2* __restrict__ Gp,
                                                    const void* __restrict__ hs, uint32_t imag_mask,
                                                    const DevState* __restrict__ st,
                                                    float2* __restrict__ vperm,
                                                    const float2* __restrict__ tw_x,
                                                    const float2* __restrict__ tw_mx) {
  if (st && st->done) return;
  extern __shared__ float2 lds[];
  const int W = g.cpw * g.nmem;
  float2* twx = lds;
  float2* twm = twx + g.nx;
  float2* U0 = twm + g.mx;
  float2* U1 = U0 + g.nx * W;
  float2* F0 = U1 + g.nx * W;
  float2* F1 = F0 + g.K * g.cpw * g.mx;
  load_table(twx, tw_x, g.nx);
  load_table(twm, tw_mx, g.mx);
  const int c0 = blockIdx.x * g.cpw;
  const int nxb = g.mx / g.xb;
  const int per_k = g.cpw * g.mx;
  for (int p = threadIdx.x; p < g.K * per_k; p += blockDim.x) {
    const int k = p / per_k, r = p % per_k;
    const int xbi = r / (g.cpw * g.xb), r2 = r % (g.cpw * g.xb);
    const int c = r2 / g.xb, xi = r2 % g.xb;
    F0[(k * g.cpw + c) * g.mx + xbi * g.xb + xi] = Gp[(((long long)k * nxb + xbi) * g.ncls + c0 + c) * g.xb + xi];
  }
  const float2* F = fft_lds<-1>(F0, F1, twm, g.mx, g.K * g.cpw, LineMap{g.K * g.cpw, 0, g.mx, 1}, false);
  const int e0 = threadIdx.x * E;
  const int per_cls = g.mx * g.S;
  const int cl = e0 / per_cls;
  const int rem = e0 % per_cls;
  const int qxp = rem / g.S;
  const int within = rem % g.S;
  float2 acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = make_float2(0.f, 0.f);
  const long long hoff0 = (long long)c0 * per_cls + e0;
  HLoad<HC, E> hc, hn;
  hc.load(hs, hoff0);
  for (int k = 0; k < g.K; ++k) {
    if (k + 1 < g.K) hn.load(hs, (long long)(k + 1) * g.hsz + hoff0);
    float2 R = F[(k * g.cpw + cl) * g.mx + qxp];
    if constexpr (HC == 0) {
      // conj(i h) R = -i h R
      if ((imag_mask >> k) & 1u) R = make_float2(R.y, -R.x);
#pragma unroll
      for (int i = 0; i < E; ++i) { acc[i].x += hc.v[i].x * R.x; acc[i].y += hc.v[i].x * R.y; }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) acc[i] = cadd(acc[i], cmulcj(hc.v[i], R));
    }
    hc = hn;
  }
  // every element of the group is written exactly once
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int w = within + i;
    const int jx = w / g.nmem, m = w % g.nmem;
    U0[(qxp + jx * g.mx) * W + cl * g.nmem + m] = acc[i];
  }
  const float2* V = fft_lds<+1>(U0, U1, twx, g.nx, W, LineMap{W, 0, 1, W}, true);
  for (int p = threadIdx.x; p < g.nx * W; p += blockDim.x) {
    const int xx = p / W, e = p % W;
    vperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e] = V[p];
  }
}

// ============================================================================ pass 3: small grid
enum { EPI_STORE = 0, EPI_RESID = 1, EPI_RESID_BACK = 2, EPI_BACK = 3 };

// 2-D R2C over (y', z') of the small-grid rows held as packed pairs in *a, then
// store the class layout G[k][xbi][class][xi].
__device__ void small_r2c_and_store(const Geo& g, float2* a, float2* b, const float2* twy, const float2* twz,
                                    float2* __restrict__ Gout, int k, int xbi) {
  const int rows = g.xb * g.my;
  float2* X = r2c_rows(a, b, twz, rows, g.mz, g.mzh, g.mzh, g.spairs);   // X[xi][class]
  float2* Y = fft_lds<-1>(X, X == a ? b : a, twy, g.my, g.xb * g.mzh, LineMap{g.mzh, g.ncls, 1, g.mzh}, true);
  const int nxb = g.mx / g.xb;
  float2* dst = Gout + ((long long)k * nxb + xbi) * g.ncls * g.xb;
  for (int p = threadIdx.x; p < g.ncls * g.xb; p += blockDim.x) {
    const int c = p / g.xb, xi = p % g.xb;
    dst[p] = Y[xi * g.ncls + c];
  }
}

// Forward pass 3 (and, with EPI_RESID_BACK / EPI_BACK, the first adjoint pass on
// the result).  grid = K * (mx/xb) blocks.  LDS: tables (my + mz) + 2 * small_lds.
template <int EPI>
__global__ __launch_bounds__(1024) void k_small_inv(Geo g, const float2* __restrict__ G,
                                                    float* __restrict__ d,
                                                    const float* __restrict__ dmeas,
                                                    const DevState* __restrict__ st,
                                                    float2* __restrict__ Gp,
                                                    const float2* __restrict__ tw_my,
                                                    const float2* __restrict__ tw_mz) {
  if (st && st->done) return;
  extern __shared__ float2 lds[];
  const int sl = small_lds(g);
  float2* twy = lds;
  float2* twz = twy + g.my;
  float2* P0 = twz + g.mz;
  float2* P1 = P0 + sl;
  load_table(twy, tw_my, g.my);
  load_table(twz, tw_mz, g.mz);
  const int nxb = g.mx / g.xb;
  const int k = blockIdx.x / nxb, xbi = blockIdx.x % nxb;
  const float2* src = G + ((long long)k * nxb + xbi) * g.ncls * g.xb;
  for (int p = threadIdx.x; p < g.ncls * g.xb; p += blockDim.x) {
    const int c = p / g.xb, xi = p % g.xb;
    P0[xi * g.ncls + c] = src[p];
  }
  float2* X = fft_lds<+1>(P0, P1, twy, g.my, g.xb * g.mzh, LineMap{g.mzh, g.ncls, 1, g.mzh}, true);
  const int rows = g.xb * g.my;
  float2* Z = c2r_rows(X, X == P0 ? P1 : P0, twz, rows, g.mz, g.mzh, g.mzh, g.spairs);
  // Z holds packed real rows: row r at pair r/2, .x (even) / .y (odd)
  float* Zf = reinterpret_cast<float*>(Z);
  const long long obase = (long long)k * g.M + (long long)xbi * g.xb * g.my * g.mz;
  const int n = rows * g.mz;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const int r = p / g.mz, z = p % g.mz;
    const int li = 2 * ((r >> 1) * g.mz + z) + (r & 1);
    const float v = Zf[li];
    if constexpr (EPI == EPI_STORE) d[obase + p] = v;
    else if constexpr (EPI == EPI_RESID) d[obase + p] = v - dmeas[obase + p];
    else if constexpr (EPI == EPI_RESID_BACK) Zf[li] = v - dmeas[obase + p];
    // EPI_BACK keeps v in place
  }
  if constexpr (EPI == EPI_RESID_BACK || EPI == EPI_BACK) {
    if (rows & 1) {
      for (int z = threadIdx.x; z < g.mz; z += blockDim.x) Zf[2 * ((rows >> 1) * g.mz + z) + 1] = 0.f;
    }
    small_r2c_and_store(g, Z, Z == P0 ? P1 : P0, twy, twz, Gp, k, xbi);
  }
}

// Adjoint pass 3: R2C of the portraits.  grid = K * (mx/xb) blocks.
__global__ __launch_bounds__(1024) void k_small_fwd(Geo g, const float* __restrict__ r,
                                                    float2* __restrict__ Gp,
                                                    const float2* __restrict__ tw_my,
                                                    const float2* __restrict__ tw_mz) {
  extern __shared__ float2 lds[];
  const int sl = small_lds(g);
  float2* twy = lds;
  float2* twz = twy + g.my;
  float2* P0 = twz + g.mz;
  float2* P1 = P0 + sl;
  load_table(twy, tw_my, g.my);
  load_table(twz, tw_mz, g.mz);
  const int nxb = g.mx / g.xb;
  const int k = blockIdx.x / nxb, xbi = blockIdx.x % nxb;
  const int rows = g.xb * g.my;
  const long long ibase = (long long)k * g.M + (long long)xbi * g.xb * g.my * g.mz;
  float* Zf = reinterpret_cast<float*>(P0);
  const int n = rows * g.mz;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const int rr = p / g.mz, z = p % g.mz;
    Zf[2 * ((rr >> 1) * g.mz + z) + (rr & 1)] = r[ibase + p];
  }
  if (rows & 1) {
    for (int z = threadIdx.x; z < g.mz; z += blockDim.x) Zf[2 * ((rows >> 1) * g.mz + z) + 1] = 0.f;
  }
  small_r2c_and_store(g, P0, P1, twy, twz, Gp, k, xbi);
}

// ============================================================================ pass 1 adjoint
enum { OUT_SCALE_B = 0, OUT_NORMAL = 1, OUT_FISTA = 2 };

// T^T T y at (x, y, z) for stacked periodic second differences: sum over axes of
// y[+2] - 4 y[+1] + 6 y - 4 y[-1] + y[-2]; reg_kind 1 gives T = I.
template <typename F>
__device__ __forceinline__ float reg_stencil(const Geo& g, int reg_kind, int x, int y, int z, F val) {
  const float c = val(x, y, z);
  if (reg_kind == 1) return c;
  auto wrap = [](int i, int n) { i %= n; return i < 0 ? i + n : i; };
  float s = 18.f * c;
  s += val(wrap(x + 2, g.nx), y, z) + val(wrap(x - 2, g.nx), y, z) - 4.f * (val(wrap(x + 1, g.nx), y, z) + val(wrap(x - 1, g.nx), y, z));
  s += val(x, wrap(y + 2, g.ny), z) + val(x, wrap(y - 2, g.ny), z) - 4.f * (val(x, wrap(y + 1, g.ny), z) + val(x, wrap(y - 1, g.ny), z));
  s += val(x, y, wrap(z + 2, g.nz)) + val(x, y, wrap(z - 2, g.nz)) - 4.f * (val(x, y, wrap(z + 1, g.nz)) + val(x, y, wrap(z - 1, g.nz)));
  return s;
}

struct AdjOut {
  float* out;              // OUT_SCALE_B / OUT_NORMAL: result
  const float* vin;        // OUT_NORMAL: w_{t-1} (v = scale * w_{t-1});  OUT_FISTA: rho^k
  const float* vprev;      // OUT_FISTA: rho^{k-1}
  float* rho_next;         // OUT_FISTA: rho^{k+1}
  double* partials;        // per-block FP64 partial sums [gridDim][2]
  DevState* st;
  int reg_kind;
  float lam;
  float* hist;             // unused placeholder
  double* hist64;          // FISTA: history of r_k indexed by (k - k_first)
  int k_first;
  int hist_len;
};

// Deterministic grid reduction: every block writes NV partials; the last block to
// arrive sums them in block order.  Returns true in thread 0 of the last block.
template <int NV>
__device__ __forceinline__ bool grid_reduce_last(double* v, double* partials, DevState* st, double* sh) {
  block_reduce_f64<NV>(v, sh);
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) partials[blockIdx.x * NV + j] = v[j];
    __threadfence();
    const int prev = atomicAdd(&st->counter, 1);
    is_last = (prev == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  if (threadIdx.x == 0) {
    __threadfence();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double s = 0.0;
      const volatile double* vp = partials;
      for (int bidx = 0; bidx < (int)gridDim.x; ++bidx) s += vp[bidx * NV + j];
      v[j] = s;
    }
    st->counter = 0;
  }
  return threadIdx.x == 0;
}

// Adjoint pass 1: gather the class layout into a half plane, inverse y FFT, C2R
// along z, then the epilogue:
//   OUT_SCALE_B  out = b . v                                  (A^T)
//   OUT_NORMAL   out = b . v + lam T^T T (s w_prev); FP64 <s w_prev, out>, ||out||^2
//   OUT_FISTA    g = b . v + lam T^T T y^k; rho^{k+1} = max(y^k - tau g, 0);
//                FP64 ||rho^{k+1} - y^k||^2, ||rho^{k+1}||^2
// grid = nx blocks.
template <int OUT>
__global__ __launch_bounds__(1024) void k_plane_adj(Geo g, const float2* __restrict__ vperm,
                                                    const float* __restrict__ b, AdjOut ao,
                                                    const float2* __restrict__ tw_y,
                                                    const float2* __restrict__ tw_z) {
  if constexpr (OUT != OUT_SCALE_B) {
    if (ao.st->done) return;
  }
  extern __shared__ float2 lds[];
  const int pl = plane_lds(g);
  float2* twz = lds;
  float2* twy = twz + g.nz;
  float2* P0 = twy + g.ny;
  float2* P1 = P0 + pl;
  __shared__ double red[64];
  load_table(twz, tw_z, g.nz);
  load_table(twy, tw_y, g.ny);
  const int x = blockIdx.x;
  const float2* src = vperm + (long long)x * g.plane;
  for (int p = threadIdx.x; p < g.ny * g.nzh; p += blockDim.x) {
    const int qy = p / g.nzh, qz = p % g.nzh;
    bool cj;
    const int e = class_index_of(g, qy, qz, cj);
    const float2 v = src[e];
    P0[p] = cj ? make_float2(v.x, -v.y) : v;
  }
  float2* X = fft_lds<+1>(P0, P1, twy, g.ny, g.nzh, LineMap{g.nzh, 0, 1, g.nzh}, true);
  float2* Z = c2r_rows(X, X == P0 ? P1 : P0, twz, g.ny, g.nz, g.nzh, g.nzh, g.npairs);
  const float* Xf = reinterpret_cast<const float*>(Z);
  const long long pbase = (long long)x * g.ny * g.nz;
  const int nyz = g.ny * g.nz;
  double acc[2] = {0.0, 0.0};
  if constexpr (OUT == OUT_SCALE_B) {
    for (int p = threadIdx.x; p < nyz; p += blockDim.x) {
      const int y = p / g.nz, z = p % g.nz;
      ao.out[pbase + p] = b[pbase + p] * Xf[2 * ((y >> 1) * g.nz + z) + (y & 1)];
    }
    return;
  } else if constexpr (OUT == OUT_NORMAL) {
    const float s = (float)ao.st->scale;
    const float* w = ao.vin;
    auto val = [&](int xx, int yy, int zz) { return s * w[((long long)xx * g.ny + yy) * g.nz + zz]; };
    for (int p = threadIdx.x; p < nyz; p += blockDim.x) {
      const int y = p / g.nz, z = p % g.nz;
      const float o = b[pbase + p] * Xf[2 * ((y >> 1) * g.nz + z) + (y & 1)] + ao.lam * reg_stencil(g, ao.reg_kind, x, y, z, val);
      ao.out[pbase + p] = o;
      acc[0] += (double)val(x, y, z) * (double)o;
      acc[1] += (double)o * (double)o;
    }
    if (grid_reduce_last<2>(acc, ao.partials, ao.st, red)) {
      DevState* st = ao.st;
      st->lmax = acc[0];
      st->scale = 1.0 / sqrt(acc[1]);
      if (!(acc[0] == acc[0]) || !(acc[1] < 1e300)) st->nonfinite = 1.0;
    }
  } else {
    DevState* st = ao.st;
    const int kk = st->k;
    const float beta = (float)((kk - 1.0) / (kk + 2.0));
    const float tau = (float)st->tau;
    const float* rk = ao.vin;
    const float* rkm1 = ao.vprev;
    auto yv = [&](int xx, int yy, int zz) {
      const long long i = ((long long)xx * g.ny + yy) * g.nz + zz;
      const float r = rk[i];
      return r + beta * (r - rkm1[i]);
    };
    double acc3[3] = {0.0, 0.0, 0.0};
    for (int p = threadIdx.x; p < nyz; p += blockDim.x) {
      const int y = p / g.nz, z = p % g.nz;
      const float yk = yv(x, y, z);
      const float gr = b[pbase + p] * Xf[2 * ((y >> 1) * g.nz + z) + (y & 1)] + ao.lam * reg_stencil(g, ao.reg_kind, x, y, z, yv);
      const float nx = fmaxf(yk - tau * gr, 0.f);
      ao.rho_next[pbase + p] = nx;
      const double dd = (double)nx - (double)yk;
      acc3[0] += dd * dd;
      acc3[1] += (double)nx * (double)nx;
      if (!isfinite(gr) || !isfinite(yk)) acc3[2] += 1.0;   // max(NaN, 0) would hide it
    }
    if (grid_reduce_last<3>(acc3, ao.partials, ao.st, red)) {
      double r;
      if (acc3[1] == 0.0) r = (acc3[0] == 0.0) ? 0.0 : __builtin_inf();
      else r = sqrt(acc3[0]) / sqrt(acc3[1]);
      st->rel_step = r;
      st->last_k = kk;
      const int hi = kk - ao.k_first;
      if (ao.hist64 && hi >= 0 && hi < ao.hist_len) ao.hist64[hi] = r;
      if (acc3[2] != 0.0 || !(acc3[0] == acc3[0]) || !(acc3[1] == acc3[1]) || acc3[1] > 1e300) {
        st->nonfinite = 1.0;
        st->done = 1;
      }
      if (r <= st->tol || kk >= st->kmax) st->done = 1;
      st->k = kk + 1;
    }
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
  const double2* F = fft_lds<-1>(X, X1, tw, nx, 1, LineMap{1, 0, nx, 1}, false);
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
  const double2* F = fft_lds<-1>(X, X1, tw, nz, 1, LineMap{1, 0, nz, 1}, false);
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
  const double2* F = fft_lds<-1>(X, X1, tw, ny, 1, LineMap{1, 0, ny, 1}, false);
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
  float2* U1 = U0 + g.nx * W;
  load_table(twx, tw_x, g.nx);
  const int c0 = blockIdx.x * g.cpw;
  for (int p = threadIdx.x; p < g.nx * W; p += blockDim.x) {
    const int xx = p / W, e = p % W;
    U0[p] = uperm[(long long)xx * g.plane + (long long)c0 * g.nmem + e];
  }
  const float2* Ul = fft_lds<-1>(U0, U1, twx, g.nx, W, LineMap{W, 0, 1, W}, true);
  const float invN = (float)(1.0 / (double)g.N);
  const int per_cls = g.mx * g.S;
  for (int t = threadIdx.x; t < g.cpw * per_cls; t += blockDim.x) {
    const int cl = t / per_cls, r2 = t % per_cls;
    const int qxp = r2 / g.S, w = r2 % g.S;
    const int jx = w / g.nmem, m = w % g.nmem;
    const float2 v = Ul[(qxp + jx * g.mx) * W + cl * g.nmem + m];
    hs[(long long)k * g.hsz + (long long)c0 * per_cls + t] = make_float2(v.x * invN, v.y * invN);
  }
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
  if (grid_reduce_last<1>(acc, partials, st, red)) st->scale = 1.0 / sqrt(acc[0]);
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
