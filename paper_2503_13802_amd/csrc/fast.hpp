// Compile-time-geometry passes of the fused operator sequences (A then A^T, the normal
// operator and the solver updates) for scalar plans with analytic (compact) spectra and
// no boundary padding, on the grids listed in the dispatch table of mh3d.hip.
//
// The operator is the same A = P H B as in kernels.hpp (Sec. 4.1 eq. dN, Table tab:ops),
// with the 3-D FFT split differently between the passes:
//
//  * The y-transform is split in two (a four-step factorisation of the length-ny DFT):
//    with y = sy*y1 + y0 and qy = q'y + my*jy,
//        Uhat(qy) = sum_y0 w_ny^(y0 q'y) w_sy^(y0 jy) V(y0, q'y),
//        V(y0, q'y) = sum_y1 u(sy*y1 + y0) w_my^(y1 q'y).
//    The plane pass runs one workgroup per (x-plane, y0): it loads the my rows
//    y = sy*y1 + y0, transforms them along z (R2C) and along y1 (length my), and stores
//    V.  The class pass, which owns all sy aliases jy of its q'y, applies the twiddles
//    w_ny^(y0 q'y) and the length-sy DFT over y0 as it loads.  The plane passes thus run
//    sy times as many workgroups, each on 1/sy of a plane.
//  * Class-layout slot (class c = (q'y, q'z), y0, jz) of x-plane x holds V(y0, q'y, qz) for
//    qz = q'z + mz*jz <= nz/2, else conj V(y0, -q'y, nz - qz) (the Hermitian partner in the
//    plane, as the full-transform layout of geo.hpp does), so the class pass applies the
//    same two steps to every slot and obtains the full-grid spectrum of each alias member.
//    The adjoint mirrors both steps: inverse length-sy DFT and conjugate twiddles in the
//    class pass, inverse length-my DFT and C2R along z in the plane pass.
//  * The fused class pass keeps each thread's spectrum elements of every harmonic in
//    registers (loaded at its start, reused by the adjoint products), so it waits on one
//    round of spectrum loads; index arithmetic is on compile-time sizes.
//
// Each call sequence runs only these passes (the slot layout above is private to them);
// the separate forward and adjoint calls, vector, padded and batched plans keep the
// passes of kernels.hpp.
#pragma once
#include "kernels.hpp"

namespace mh3d {

template <int NX_, int NY_, int NZ_, int SX_, int SY_, int SZ_, int E_, int CPW_, int KMAX_>
struct FastGeo {
  static constexpr int NX = NX_, NY = NY_, NZ = NZ_, SX = SX_, SY = SY_, SZ = SZ_;
  static constexpr int MX = NX / SX, MY = NY / SY, MZ = NZ / SZ;
  static constexpr int NZH = NZ / 2 + 1, MZH = MZ / 2 + 1;
  static constexpr int NMEM = SY * SZ, S = SX * SY * SZ, NCLS = MY * MZH, PLANE = NCLS * NMEM;
  static constexpr long long HSZ = (long long)PLANE * NX;   // spectrum elements per harmonic
  static constexpr int E = E_, CPW = CPW_, KMAX = KMAX_;
  static constexpr int LG = S / E;                          // threads of one fold group
  static constexpr int TC = CPW * MX * S / E;               // class-pass threads
  static constexpr int W = CPW * NMEM;                      // member lines of a class block
  static constexpr int LSX = NX | 1, LSZ = NZ | 1, LSY = MY | 1;
  static constexpr int NP = MY / 2;                         // row pairs of a plane block
  static constexpr int TP = 256;                            // plane-pass threads
  static constexpr int NBP = NX * SY;                       // plane-pass blocks
  // one plane-pass LDS buffer: packed row pairs, half-spectrum columns or the staged slots
  static constexpr int PB0 = NP * LSZ, PB1 = NZH * LSY, PB2 = NCLS * SZ;
  static constexpr int PBUF = PB0 > PB1 ? (PB0 > PB2 ? PB0 : PB2) : (PB1 > PB2 ? PB1 : PB2);
  static constexpr size_t LDS_PLANE = sizeof(float2) * (NZ + MY + 2 * (size_t)PBUF);
  static constexpr size_t LDS_CLASS = sizeof(float2) * (NX + MX + 2 * (size_t)W * LSX + 2 * (size_t)KMAX * CPW * MX
                                                        + (size_t)CPW * SY);
  static_assert(MY % 2 == 0, "row pairs: my must be even");
  static_assert((NZ % 4) == 0, "rows are loaded as float4");
  static_assert(S % E == 0 && (LG & (LG - 1)) == 0 && LG <= 64, "fold groups are aligned lane groups");
  static_assert(NCLS % CPW == 0, "classes per block must divide the classes");
  static_assert(TC <= 1024, "class block too large");
  static_assert(SY == 1 || SY == 2 || SY == 4 || SY == 3, "length-sy DFT");
};

// Plane-pass block b -> (x-plane, y0).  The blocks of one XCD (b mod 8) take a run of
// consecutive planes with all their y0, so the sy blocks that complete one plane's slots
// and the stencil's neighbouring planes share that XCD's L2.
template <class G>
__device__ __forceinline__ void fast_plane_of(int b, int& x, int& y0) {
  if constexpr (G::NX % 8 == 0) {
    const int i = b >> 3;
    y0 = i % G::SY;
    x = (b & 7) * (G::NX / 8) + i / G::SY;
  } else {
    y0 = b % G::SY;
    x = b / G::SY;
  }
}

// Sum over aligned groups of LG lanes (every lane of a group gets the group's sum).
// Lane groups of up to 16 use DPP moves inside a row; wider groups use shuffles.
template <int LG>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (LG >= 2) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  if constexpr (LG >= 4) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  if constexpr (LG >= 8) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  if constexpr (LG >= 16) v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false));
  if constexpr (LG >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (LG >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// ============================================================================ plane pass (forward)
// Block (x, y0): u = b . a on rows y = sy*y1 + y0 of plane x (a: rho, y^k or s w by SRC),
// R2C along z, length-my DFT along y1, slots stored for the class pass.
template <class G, int SRC>
__global__ __launch_bounds__(256) void k_fast_plane_fwd(const VolDesc* __restrict__ vds, const float* __restrict__ a) {
  const VolDesc& vd = vds[0];
  if constexpr (SRC == SRC_FISTA_Y || SRC == SRC_SCALED) {
    if (vd.st->done) return;
  }
  if constexpr (SRC == SRC_FISTA_Y) a = vd.y[vd.st->k & 1];
  if constexpr (SRC == SRC_SCALED) {
    if (!a) a = vd.rho[vd.st->k & 1];
  }
  int x, y0;
  fast_plane_of<G>(blockIdx.x, x, y0);
  extern __shared__ float2 lds[];
  float2* twz = lds;
  float2* twy = twz + G::NZ;
  float2* B0 = twy + G::MY;
  float2* B1 = B0 + G::PBUF;
  constexpr int F4R = G::NZ / 4, F4 = G::MY * F4R, NL = (F4 + G::TP - 1) / G::TP;
  const long long pb = (long long)x * G::NY * G::NZ;
  const float* __restrict__ bs = vd.b;
  float4 va[NL], vb[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int f = threadIdx.x + G::TP * i;
    if (f < F4) {
      const int y1 = f / F4R, c4 = f - (f / F4R) * F4R;
      const long long off = pb + (long long)(G::SY * y1 + y0) * G::NZ + 4 * c4;
      va[i] = *reinterpret_cast<const float4*>(a + off);
      vb[i] = *reinterpret_cast<const float4*>(bs + off);
    }
  }
  load_table(twz, vd.tw + vd.off[2], G::NZ);
  load_table(twy, vd.tw + vd.off[4], G::MY);
  float c = 1.f;
  if constexpr (SRC == SRC_SCALED) c = (float)vd.st->scale;
  float* Zf = reinterpret_cast<float*>(B0);
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int f = threadIdx.x + G::TP * i;
    if (f < F4) {
      const int y1 = f / F4R, c4 = f - (f / F4R) * F4R;
      float u[4];
      const float av[4] = {va[i].x, va[i].y, va[i].z, va[i].w};
      const float bv[4] = {vb[i].x, vb[i].y, vb[i].z, vb[i].w};
#pragma unroll
      for (int q = 0; q < 4; ++q) u[q] = (SRC == SRC_SCALED) ? bv[q] * (c * av[q]) : bv[q] * av[q];
      float* row = Zf + 2 * ((y1 >> 1) * G::LSZ + 4 * c4) + (y1 & 1);
#pragma unroll
      for (int q = 0; q < 4; ++q) row[2 * q] = u[q];
    }
  }
  __syncthreads();
  float2* Z = ct_stages<G::NZ, 0, 1, -1>(B0, B1, twz, G::NP, G::LSZ);
  float2* X = (Z == B0) ? B1 : B0;
  // split each packed pair into its two half spectra, columns X[qz][y1]
  for (int it = threadIdx.x; it < G::NP * G::NZH; it += G::TP) {
    const int j = it / G::NZH, q = it - (it / G::NZH) * G::NZH;
    const float2 zq = Z[j * G::LSZ + q];
    const float2 zm = Z[j * G::LSZ + (q == 0 ? 0 : G::NZ - q)];
    X[q * G::LSY + 2 * j] = make_float2(0.5f * (zq.x + zm.x), 0.5f * (zq.y - zm.y));
    X[q * G::LSY + 2 * j + 1] = make_float2(0.5f * (zq.y + zm.y), -0.5f * (zq.x - zm.x));
  }
  __syncthreads();
  const float2* Y = ct_stages<G::MY, 0, 1, -1>(X, Z, twy, G::NZH, G::LSY);
  // slots of plane x for this y0: class c, members jz (SZ consecutive complex)
  float2* __restrict__ dst = vd.uperm + (long long)x * G::PLANE + y0 * G::SZ;
  for (int c = threadIdx.x; c < G::NCLS; c += G::TP) {
    const int qyp = c / G::MZH, qzp = c - (c / G::MZH) * G::MZH;
    float2 v[G::SZ];
#pragma unroll
    for (int jz = 0; jz < G::SZ; ++jz) {
      const int qz = qzp + G::MZ * jz;
      if (2 * qz <= G::NZ) {
        v[jz] = Y[qz * G::LSY + qyp];
      } else {
        const float2 w = Y[(G::NZ - qz) * G::LSY + (qyp == 0 ? 0 : G::MY - qyp)];
        v[jz] = make_float2(w.x, -w.y);
      }
    }
    float2* o = dst + (long long)c * G::NMEM;
    if constexpr (G::SZ % 2 == 0) {
#pragma unroll
      for (int jz = 0; jz < G::SZ; jz += 2)
        *reinterpret_cast<float4*>(o + jz) = make_float4(v[jz].x, v[jz].y, v[jz + 1].x, v[jz + 1].y);
    } else {
#pragma unroll
      for (int jz = 0; jz < G::SZ; ++jz) o[jz] = v[jz];
    }
  }
}

// ============================================================================ class pass (fused)
// Forward products of the block's classes (spectrum Hhat_k times the alias members,
// folded), then from those folded spectra the adjoint products (sum over k of
// conj(Hhat_k) times the tiled residual), as class_normal_body does; mode NRM_RESID
// subtracts the data's spectra (G'), NRM_STORE also writes the portraits' decimated
// spectra G for the small-grid pass.
template <class G, int MODE>
__global__ __launch_bounds__(G::TC) void k_fast_class(const VolDesc* __restrict__ vds, int check_done) {
  const VolDesc& vd = vds[0];
  if (check_done && vd.st->done) return;
  constexpr int NX = G::NX, MX = G::MX, S = G::S, E = G::E, NMEM = G::NMEM, SY = G::SY, SZ = G::SZ;
  constexpr int LSX = G::LSX, W = G::W, CPW = G::CPW, KMAX = G::KMAX;
  const int lb = plane_of_block(blockIdx.x, gridDim.x);
  const int c0 = lb * CPW;
  const int K = vd.g.K;
  extern __shared__ float2 lds[];
  float2* twx = lds;
  float2* twm = twx + NX;
  float2* U0 = twm + MX;
  float2* U1 = U0 + W * LSX;
  float2* F0 = U1 + W * LSX;
  float2* F1 = F0 + KMAX * CPW * MX;
  float2* twc = F1 + KMAX * CPW * MX;   // [cl][y0]: w_ny^(y0 q'y) of each class
  const int t = threadIdx.x;
  const int e0 = t * E;
  const int cl = e0 / (MX * S);
  const int rem = e0 - cl * (MX * S);
  const int qxp = rem / S;
  const int within = rem - qxp * S;
  // every harmonic's spectra of this thread's elements (contiguous: [k][class][q'x][jx][member])
  HLoad<0, E> hb[KMAX];
  const long long hoff0 = (long long)c0 * MX * S + e0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < K) hb[k].load(vd.hs, (long long)k * G::HSZ + hoff0);
  if constexpr (MODE == NRM_RESID) {
    const float2* __restrict__ Dt = vd.Gp;
    for (int p = t; p < K * CPW * MX; p += G::TC) {
      const int k = p / (CPW * MX), r = p - k * (CPW * MX);
      F1[p] = Dt[((long long)k * G::NCLS + c0) * MX + r];
    }
  }
  load_table(twx, vd.tw + vd.off[0], NX);
  load_table(twm, vd.tw + vd.off[3], MX);
  if constexpr (SY > 1) {
    for (int p = t; p < CPW * SY; p += G::TC) {
      const int c = p / SY, y0 = p - c * SY;
      const int qyp = (c0 + c) / G::MZH;
      twc[p] = vd.tw[vd.off[1] + (y0 * qyp) % G::NY];
    }
    __syncthreads();
  }
  // slots -> alias members: twiddle and length-sy DFT over y0 at each (x, jz)
  const float2* __restrict__ up = vd.uperm;
  constexpr int NIT = CPW * NX * SZ;
  for (int it = t; it < NIT; it += G::TC) {
    const int c = it / (NX * SZ), r = it - c * (NX * SZ);
    const int xx = r / SZ, jz = r - (r / SZ) * SZ;
    const float2* src = up + (long long)xx * G::PLANE + (long long)(c0 + c) * NMEM + jz;
    float2 v[SY];
#pragma unroll
    for (int y0 = 0; y0 < SY; ++y0) v[y0] = src[y0 * SZ];
    if constexpr (SY > 1) {
#pragma unroll
      for (int y0 = 1; y0 < SY; ++y0) v[y0] = cmul(v[y0], twc[c * SY + y0]);
      dft<SY, -1>(v);
    }
#pragma unroll
    for (int jy = 0; jy < SY; ++jy) U0[(c * NMEM + jy * SZ + jz) * LSX + xx] = v[jy];
  }
  __syncthreads();
  const float2* U = ct_stages<NX, 0, 1, -1>(U0, U1, twx, W, LSX);
  float2 ur[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int w = within + i;
    const int jx = w / NMEM, m = w - (w / NMEM) * NMEM;
    ur[i] = U[(cl * NMEM + m) * LSX + qxp + jx * MX];
  }
  const uint32_t imag_mask = vd.imag_mask;
  const bool lead = (t & (G::LG - 1)) == 0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      float ax = 0.f, ay = 0.f;
#pragma unroll
      for (int i = 0; i < E; ++i) { ax += hb[k].v[i] * ur[i].x; ay += hb[k].v[i] * ur[i].y; }
      ax = group_sum<G::LG>(ax);
      ay = group_sum<G::LG>(ay);
      if (lead) F0[(k * CPW + cl) * MX + qxp] = ((imag_mask >> k) & 1u) ? make_float2(-ay, ax) : make_float2(ax, ay);
    }
  }
  __syncthreads();   // Fhat complete; the member lines are free
  const float Mf = (float)(G::MX * G::MY * G::MZ);
  float2 acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      const int fi = (k * CPW + cl) * MX + qxp;
      const float2 f = F0[fi];
      float2 R = make_float2(Mf * f.x, Mf * f.y);
      if constexpr (MODE == NRM_RESID) R = csub(R, F1[fi]);
      if ((imag_mask >> k) & 1u) R = make_float2(R.y, -R.x);   // conj(i h) R = -i h R
#pragma unroll
      for (int i = 0; i < E; ++i) { acc[i].x += hb[k].v[i] * R.x; acc[i].y += hb[k].v[i] * R.y; }
    }
  }
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int w = within + i;
    const int jx = w / NMEM, m = w - (w / NMEM) * NMEM;
    U0[(cl * NMEM + m) * LSX + qxp + jx * MX] = acc[i];
  }
  __syncthreads();
  const float2* V = ct_stages<NX, 0, 1, +1>(U0, U1, twx, W, LSX);
  // alias members -> slots: inverse length-sy DFT over jy, conjugate twiddles
  float2* __restrict__ vp = vd.uperm;
  for (int it = t; it < NIT; it += G::TC) {
    const int c = it / (NX * SZ), r = it - c * (NX * SZ);
    const int xx = r / SZ, jz = r - (r / SZ) * SZ;
    float2 v[SY];
#pragma unroll
    for (int jy = 0; jy < SY; ++jy) v[jy] = V[(c * NMEM + jy * SZ + jz) * LSX + xx];
    if constexpr (SY > 1) {
      dft<SY, +1>(v);
#pragma unroll
      for (int y0 = 1; y0 < SY; ++y0) v[y0] = cmulcj(twc[c * SY + y0], v[y0]);
    }
    float2* dst = vp + (long long)xx * G::PLANE + (long long)(c0 + c) * NMEM + jz;
#pragma unroll
    for (int y0 = 0; y0 < SY; ++y0) dst[y0 * SZ] = v[y0];
  }
  if constexpr (MODE == NRM_STORE) {
    const float2* F = ct_stages<MX, 0, 1, +1>(F0, F1, twm, K * CPW, MX);
    float2* __restrict__ Gs = vd.G;
    const Geo& g = vd.g;
    const int xb = g.xb, nxb = MX / xb;
    for (int p = t; p < K * CPW * MX; p += G::TC) {
      const int k = p / (CPW * MX), r = p - k * (CPW * MX);
      const int xbi = r / (CPW * xb), r2 = r - xbi * (CPW * xb);
      const int c = r2 / xb, xi = r2 - c * xb;
      Gs[(((long long)k * nxb + xbi) * G::NCLS + c0 + c) * xb + xi] = F[(k * CPW + c) * MX + xbi * xb + xi];
    }
  }
}

// ============================================================================ plane pass (adjoint)
// Block (x, y0): gather this y0's slots into the half spectrum, inverse length-my DFT
// along y1, C2R along z, then per voxel of rows y = sy*y1 + y0:
//   OUT_SCALE_B      ao.out = b . v
//   OUT_STEP_NORMAL  / OUT_STEP_FISTA: the solver step with u = b . v (StepCtx), FP64
//                    block partials in vd.partials[lb] for k_vol_finish (nb_upd = NBP).
template <class G, int OUT>
__device__ __forceinline__ void fast_plane_adj_body(const VolDesc& vd, int lb, const AdjOut& ao) {
  constexpr bool kStep = (OUT == OUT_STEP_NORMAL || OUT == OUT_STEP_FISTA);
  if constexpr (kStep) {
    if (vd.st->done) return;
  }
  int x, y0;
  fast_plane_of<G>(lb, x, y0);
  extern __shared__ float2 lds[];
  float2* twz = lds;
  float2* twy = twz + G::NZ;
  float2* B0 = twy + G::MY;
  float2* B1 = B0 + G::PBUF;
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  // this y0's slots of every class, staged in B1 as [class][jz]
  {
    const float2* __restrict__ src = vd.uperm + (long long)x * G::PLANE + y0 * G::SZ;
    if constexpr (G::SZ % 2 == 0) {
      constexpr int H = G::SZ / 2, N4 = G::NCLS * H;
      batched<4, float4>(N4,
                         [&](int p) {
                           const int c = p / H, h = p - (p / H) * H;
                           return *reinterpret_cast<const float4*>(src + (long long)c * G::NMEM + 2 * h);
                         },
                         [&](int p, float4 v) {
                           const int c = p / H, h = p - (p / H) * H;
                           B1[c * G::SZ + 2 * h] = make_float2(v.x, v.y);
                           B1[c * G::SZ + 2 * h + 1] = make_float2(v.z, v.w);
                         });
    } else {
      batched<4, float2>(G::NCLS * G::SZ,
                         [&](int p) { return src[(long long)(p / G::SZ) * G::NMEM + p % G::SZ]; },
                         [&](int p, float2 v) { B1[p] = v; });
    }
  }
  load_table(twz, vd.tw + vd.off[2], G::NZ);
  load_table(twy, vd.tw + vd.off[4], G::MY);
  __syncthreads();
  // half spectrum, columns B0[qz][q'y]: slot of the class holding (q'y, qz) directly, or
  // the conjugate of the Hermitian partner's slot
  for (int it = t; it < G::NZH * G::MY; it += nt) {
    const int qz = it / G::MY, qyp = it - (it / G::MY) * G::MY;
    const int qzr = qz % G::MZ;
    float2 v;
    if (2 * qzr <= G::MZ) {
      v = B1[(qyp * G::MZH + qzr) * G::SZ + qz / G::MZ];
    } else {
      const int qzm = G::NZ - qz;   // the partner's member, > nz/2
      const int cy = qyp == 0 ? 0 : G::MY - qyp;
      const float2 w = B1[(cy * G::MZH + qzm % G::MZ) * G::SZ + qzm / G::MZ];
      v = make_float2(w.x, -w.y);
    }
    B0[qz * G::LSY + qyp] = v;
  }
  __syncthreads();
  float2* X = ct_stages<G::MY, 0, 1, +1>(B0, B1, twy, G::NZH, G::LSY);
  float2* Zb = (X == B0) ? B1 : B0;
  // C2R along z: packed rows Z[j] = X[2j] + i X[2j+1] with the Hermitian extension
  for (int it = t; it < G::NP * G::NZ; it += nt) {
    const int j = it / G::NZ, q = it - (it / G::NZ) * G::NZ;
    const bool upper = 2 * q > G::NZ;
    const int qq = upper ? G::NZ - q : q;
    float2 xv = X[qq * G::LSY + 2 * j];
    float2 yv = X[qq * G::LSY + 2 * j + 1];
    if (qq == 0 || 2 * qq == G::NZ) { xv.y = 0.f; yv.y = 0.f; }
    if (upper) { xv.y = -xv.y; yv.y = -yv.y; }
    Zb[j * G::LSZ + q] = make_float2(xv.x - yv.y, xv.y + yv.x);
  }
  __syncthreads();
  const float2* Z = ct_stages<G::NZ, 0, 1, +1>(Zb, X, twz, G::NP, G::LSZ);
  const float* Zf = reinterpret_cast<const float*>(Z);
  const long long pb = (long long)x * G::NY * G::NZ;
  const float* __restrict__ bs = vd.b;
  constexpr int F4R = G::NZ / 4, F4 = G::MY * F4R;
  if constexpr (!kStep) {
    float* __restrict__ out = ao.out;
    batched<4, float4>(F4,
                       [&](int f) {
                         const int y1 = f / F4R, c4 = f - (f / F4R) * F4R;
                         return *reinterpret_cast<const float4*>(bs + pb + (long long)(G::SY * y1 + y0) * G::NZ + 4 * c4);
                       },
                       [&](int f, float4 bv) {
                         const int y1 = f / F4R, c4 = f - (f / F4R) * F4R;
                         const float* zr = Zf + 2 * ((y1 >> 1) * G::LSZ + 4 * c4) + (y1 & 1);
                         *reinterpret_cast<float4*>(out + pb + (long long)(G::SY * y1 + y0) * G::NZ + 4 * c4) =
                             make_float4(bv.x * zr[0], bv.y * zr[2], bv.z * zr[4], bv.w * zr[6]);
                       });
  } else {
    constexpr int UPD = OUT == OUT_STEP_NORMAL ? UPD_NORMAL : UPD_FISTA;
    constexpr int NV = StepCtx<UPD>::NV;
    __shared__ double red[64];
    const StepCtx<UPD> ctx(vd, ao);
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    constexpr int n = G::MY * G::NZ;
    constexpr int U = 3;
    for (int p = t; p < n; p += U * G::TP) {
      StencilVals v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int pq = p + q * G::TP;
        if (pq < n) {
          const int y1 = pq / G::NZ, z = pq - (pq / G::NZ) * G::NZ;
          const long long i = pb + (long long)(G::SY * y1 + y0) * G::NZ + z;
          v[q] = ctx.load(i, __fmul_rn(bs[i], Zf[2 * ((y1 >> 1) * G::LSZ + z) + (y1 & 1)]));
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int pq = p + q * G::TP;
        if (pq < n) {
          const int y1 = pq / G::NZ, z = pq - (pq / G::NZ) * G::NZ;
          ctx.apply(pb + (long long)(G::SY * y1 + y0) * G::NZ + z, v[q], acc);
        }
      }
    }
    store_step_partials<NV>(vd, acc, red, lb);
  }
}

template <class G, int OUT>
__global__ __launch_bounds__(256) void k_fast_plane_adj(const VolDesc* __restrict__ vds, AdjOut ao) {
  fast_plane_adj_body<G, OUT>(vds[0], blockIdx.x, ao);
}

// A then A^T after k_fast_class<NRM_STORE>: blocks [0, NBP) run the adjoint plane pass
// (ao.out = b . v), the others the small-grid inverse pass that writes the portraits d.
template <class G>
__global__ __launch_bounds__(256) void k_fast_adj_and_store(const VolDesc* __restrict__ vds, AdjOut ao,
                                                            float* __restrict__ d) {
  const VolDesc& vd = vds[0];
  if ((int)blockIdx.x < G::NBP) fast_plane_adj_body<G, OUT_SCALE_B>(vd, blockIdx.x, ao);
  else small_inv_body<EPI_STORE>(vd, blockIdx.x - G::NBP, d);
}

}  // namespace mh3d
