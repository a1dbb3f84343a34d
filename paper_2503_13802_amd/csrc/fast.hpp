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

// Stockham stages of NL lines of length N held at l*LS + p (LS odd) with consecutive
// lanes on consecutive lines (the same butterfly of each): with an odd line stride the
// strided stores of a stage fall in distinct banks, and the lanes of a butterfly
// position share its twiddles (one broadcast read).
template <int N, int R, int NS, int SGN, int NL, int LS>
__device__ __forceinline__ void lf_stage(const float2* __restrict__ in, float2* __restrict__ out, const float2* tw) {
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
  constexpr int total = NL * NB;
  for (int b = threadIdx.x; b < total; b += blockDim.x) {
    const int l = b % NL, j = b / NL;
    const int k = j % NS;
    const int base = l * LS;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[base + j + r * NB];
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[k * r * TWS];
        v[r] = SGN < 0 ? cmul(v[r], w) : cmulcj(w, v[r]);
      }
    }
    dft<R, SGN>(v);
    const int o = base + (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[o + r * NS] = v[r];
  }
}

// Length-N transforms (unnormalised) of NL lines in *a, ping-ponging with *b; a barrier
// ends each stage.  Returns the buffer holding the result.  No leading barrier.
template <int N, int S, int NS, int SGN, int NL, int LS>
__device__ __forceinline__ float2* lf_fft(float2* a, float2* b, const float2* tw) {
  constexpr int R = ct_radix(N, S);
  if constexpr (R == 0) {
    return a;
  } else {
    lf_stage<N, R, NS, SGN, NL, LS>(a, b, tw);
    __syncthreads();
    return lf_fft<N, S + 1, NS * R, SGN, NL, LS>(b, a, tw);
  }
}

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
  // items (row pair j, 4 columns): rows 2j and 2j+1 of the block (y = sy*y1 + y0) become
  // the real and imaginary parts of packed line j
  constexpr int F4R = G::NZ / 4, F4 = G::NP * F4R, NL = (F4 + G::TP - 1) / G::TP;
  const long long pb = (long long)x * G::NY * G::NZ;
  const float* __restrict__ bs = vd.b;
  float4 va[NL][2], vb[NL][2];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int f = threadIdx.x + G::TP * i;
    if (f < F4) {
      const int j = f / F4R, c4 = f - (f / F4R) * F4R;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const long long off = pb + (long long)(G::SY * (2 * j + h) + y0) * G::NZ + 4 * c4;
        va[i][h] = *reinterpret_cast<const float4*>(a + off);
        vb[i][h] = *reinterpret_cast<const float4*>(bs + off);
      }
    }
  }
  load_table(twz, vd.tw + vd.off[2], G::NZ);
  load_table(twy, vd.tw + vd.off[4], G::MY);
  float c = 1.f;
  if constexpr (SRC == SRC_SCALED) c = (float)vd.st->scale;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int f = threadIdx.x + G::TP * i;
    if (f < F4) {
      const int j = f / F4R, c4 = f - (f / F4R) * F4R;
      float u[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float av[4] = {va[i][h].x, va[i][h].y, va[i][h].z, va[i][h].w};
        const float bv[4] = {vb[i][h].x, vb[i][h].y, vb[i][h].z, vb[i][h].w};
#pragma unroll
        for (int q = 0; q < 4; ++q) u[h][q] = (SRC == SRC_SCALED) ? bv[q] * (c * av[q]) : bv[q] * av[q];
      }
      float4* dst4 = reinterpret_cast<float4*>(B0 + j * G::LSZ + 4 * c4);
      if constexpr (G::LSZ % 2 == 0) {
        dst4[0] = make_float4(u[0][0], u[1][0], u[0][1], u[1][1]);
        dst4[1] = make_float4(u[0][2], u[1][2], u[0][3], u[1][3]);
      } else {
        float2* d2 = B0 + j * G::LSZ + 4 * c4;
#pragma unroll
        for (int q = 0; q < 4; ++q) d2[q] = make_float2(u[0][q], u[1][q]);
      }
    }
  }
  __syncthreads();
  float2* Z = lf_fft<G::NZ, 0, 1, -1, G::NP, G::LSZ>(B0, B1, twz);
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
  const float2* Y = lf_fft<G::MY, 0, 1, -1, G::NZH, G::LSY>(X, Z, twy);
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
  // Issue order matters: vector-memory counters retire in order, so a wait for a load
  // also waits for every load issued before it.  Small tables and the data term first,
  // then the slot loads, then the spectra (not needed until after the x transform), so
  // the transform runs while the spectra stream in.
  load_table(twx, vd.tw + vd.off[0], NX);
  load_table(twm, vd.tw + vd.off[3], MX);
  if constexpr (MODE == NRM_RESID) {
    const float2* __restrict__ Dt = vd.Gp;
    for (int p = t; p < K * CPW * MX; p += G::TC) {
      const int k = p / (CPW * MX), r = p - k * (CPW * MX);
      F1[p] = Dt[((long long)k * G::NCLS + c0) * MX + r];
    }
  }
  if constexpr (SY > 1) {
    for (int p = t; p < CPW * SY; p += G::TC) {
      const int c = p / SY, y0 = p - c * SY;
      const int qyp = (c0 + c) / G::MZH;
      twc[p] = vd.tw[vd.off[1] + (y0 * qyp) % G::NY];
    }
    __syncthreads();
  }
  // slots (y0, jz) of the block's classes at each x, into registers
  const float2* __restrict__ up = vd.uperm;
  constexpr int NIT = CPW * NX * SZ;
  constexpr int NI = (NIT + G::TC - 1) / G::TC;
  float2 sv[NI][SY];
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int it = t + i * G::TC;
    if (NIT % G::TC == 0 || it < NIT) {
      const int c = it / (NX * SZ), r = it - c * (NX * SZ);
      const int xx = r / SZ, jz = r - (r / SZ) * SZ;
      const float2* src = up + (long long)xx * G::PLANE + (long long)(c0 + c) * NMEM + jz;
#pragma unroll
      for (int y0 = 0; y0 < SY; ++y0) sv[i][y0] = src[y0 * SZ];
    }
  }
  // every harmonic's spectra of this thread's elements (contiguous: [k][class][q'x][jx][member])
  HLoad<0, E> hb[KMAX];
  const long long hoff0 = (long long)c0 * MX * S + e0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < K) hb[k].load(vd.hs, (long long)k * G::HSZ + hoff0);
  // slots -> alias members: twiddle and length-sy DFT over y0 at each (x, jz)
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int it = t + i * G::TC;
    if (NIT % G::TC == 0 || it < NIT) {
      const int c = it / (NX * SZ), r = it - c * (NX * SZ);
      const int xx = r / SZ, jz = r - (r / SZ) * SZ;
      float2* v = sv[i];
      if constexpr (SY > 1) {
#pragma unroll
        for (int y0 = 1; y0 < SY; ++y0) v[y0] = cmul(v[y0], twc[c * SY + y0]);
        dft<SY, -1>(v);
      }
#pragma unroll
      for (int jy = 0; jy < SY; ++jy) U0[(c * NMEM + jy * SZ + jz) * LSX + xx] = v[jy];
    }
  }
  __syncthreads();
  const float2* U = lf_fft<NX, 0, 1, -1, W, LSX>(U0, U1, twx);
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
  const float2* V = lf_fft<NX, 0, 1, +1, W, LSX>(U0, U1, twx);
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
  // this y0's slots of every class, staged in B1 as [class][jz]; every load is issued
  // before the first is used (and, for A^T, the sensitivity rows of the output too)
  const long long pb = (long long)x * G::NY * G::NZ;
  const float* __restrict__ bs = vd.b;
  constexpr int F4R = G::NZ / 4, P4 = G::NP * F4R, NB4 = (P4 + G::TP - 1) / G::TP;
  float4 bq[kStep ? 1 : NB4][2];
  {
    const float2* __restrict__ src = vd.uperm + (long long)x * G::PLANE + y0 * G::SZ;
    static_assert(G::SZ % 2 == 0, "slots are loaded in pairs");
    constexpr int H = G::SZ / 2, N4 = G::NCLS * H, NS4 = (N4 + G::TP - 1) / G::TP;
    float4 sl[NS4];
#pragma unroll
    for (int i = 0; i < NS4; ++i) {
      const int p = t + i * G::TP;
      if (p < N4) {
        const int c = p / H, h = p - (p / H) * H;
        sl[i] = *reinterpret_cast<const float4*>(src + (long long)c * G::NMEM + 2 * h);
      }
    }
    if constexpr (!kStep) {
#pragma unroll
      for (int i = 0; i < NB4; ++i) {
        const int f = t + i * G::TP;
        if (f < P4) {
          const int j = f / F4R, c4 = f - (f / F4R) * F4R;
          const long long o0 = pb + (long long)(G::SY * 2 * j + y0) * G::NZ + 4 * c4;
          bq[i][0] = *reinterpret_cast<const float4*>(bs + o0);
          bq[i][1] = *reinterpret_cast<const float4*>(bs + o0 + (long long)G::SY * G::NZ);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NS4; ++i) {
      const int p = t + i * G::TP;
      if (p < N4) {
        const int c = p / H, h = p - (p / H) * H;
        B1[c * G::SZ + 2 * h] = make_float2(sl[i].x, sl[i].y);
        B1[c * G::SZ + 2 * h + 1] = make_float2(sl[i].z, sl[i].w);
      }
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
  float2* X = lf_fft<G::MY, 0, 1, +1, G::NZH, G::LSY>(B0, B1, twy);
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
  const float2* Z = lf_fft<G::NZ, 0, 1, +1, G::NP, G::LSZ>(Zb, X, twz);
  const float* Zf = reinterpret_cast<const float*>(Z);
  if constexpr (!kStep) {
    // items (row pair j, 4 columns): packed line j holds rows 2j (real) and 2j+1 (imaginary)
    float* __restrict__ out = ao.out;
#pragma unroll
    for (int i = 0; i < NB4; ++i) {
      const int f = t + i * G::TP;
      if (f >= P4) break;
      const int j = f / F4R, c4 = f - (f / F4R) * F4R;
      const long long o0 = pb + (long long)(G::SY * 2 * j + y0) * G::NZ + 4 * c4;
      const long long o1 = o0 + (long long)G::SY * G::NZ;
      const float4 b0 = bq[i][0], b1 = bq[i][1];
      const float2* zr = Z + j * G::LSZ + 4 * c4;
      const float2 z0 = zr[0], z1 = zr[1], z2 = zr[2], z3 = zr[3];
      *reinterpret_cast<float4*>(out + o0) = make_float4(b0.x * z0.x, b0.y * z1.x, b0.z * z2.x, b0.w * z3.x);
      *reinterpret_cast<float4*>(out + o1) = make_float4(b1.x * z0.y, b1.y * z1.y, b1.z * z2.y, b1.w * z3.y);
    }
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
