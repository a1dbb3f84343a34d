// Compile-time-geometry passes of the fused operator sequences (A then A^T, the normal
// operator and the solver updates) for scalar plans with the analytic PSF and no
// boundary padding, on the grids listed in the dispatch table of mh3d.hip.
//
// They compute the operator A = P H B of kernels.hpp (Sec. 4.1 eq. dN, Table tab:ops)
// through two factorisations:
//
//  * The analytic PSF is separable, h_k(x, y, z) = c_k L^(k)(a x) E(y, z) (Sec. 3.3
//    eq. hkapprox), so Hhat_k(qx, qy, qz) = F_k(qx) Ehat(qy, qz).  The transverse factor
//    is common to every harmonic: A_k u = P_x [ f_k (*)_x P_yz [ E (*)_yz u ] ].  The plane
//    passes apply Ehat and fold the (y, z) aliases of each x-plane (P_yz in Fourier form),
//    leaving my (mz/2 + 1) values per plane; the column pass transforms each of these
//    columns along x, multiplies by every F_k and folds the x aliases.  The spectra are
//    never stored: K nx + sy my (nz/2 + 1) numbers replace K nx ny (nz/2 + 1).  Ehat is
//    real and even in qy and qz (E is even in y and z with the symmetric sampling of the
//    even-length midpoint), F_k is real for odd derivative orders and imaginary for even.
//  * The y-transform is split four-step: with y = sy*y1 + y0 and qy = q'y + my*jy,
//        Uhat(qy) = sum_y0 w_ny^(y0 qy) V(y0, q'y),  V(y0, q'y) = sum_y1 u(sy*y1 + y0) w_my^(y1 q'y),
//    so the Ehat-weighted fold over jy of one residue y0 is V(y0, q'y) times
//        Et(y0, q'y, qz) = sum_jy w_ny^(y0 qy) Ehat(qy, qz)   (a plan-time table).
//    Each plane workgroup takes one (x-plane, y0): it loads the my rows y = sy*y1 + y0,
//    transforms them along z (R2C) and y1, and writes its share of the folded plane,
//        C(y0; x, q'y, q'z) = sum_jz Et(y0, q'y, qz) V(y0, q'y, qz),  qz = q'z + mz*jz,
//    (for qz > nz/2 the Hermitian partner conj V(y0, -q'y, nz - qz), Et even in qz); the
//    column pass sums the sy shares.  The adjoint mirrors it: the column pass leaves Q(x,
//    q'y, q'z) = x-transform of sum_k conj(F_k) R_k, and plane workgroup (x, y0) forms
//    the residue's spectrum Q(x, q'y, qz mod mz) conj(Et(y0, q'y, qz)) (Q Hermitian in
//    (q'y, q'z) for the q'z beyond mz/2), transforms it back along y1 and z (C2R) and
//    multiplies by b.
//
// Each call sequence runs only these passes (their intermediate layouts are their own):
// the fused sequences, the separate forward and adjoint calls and the per-harmonic
// back-projections (the adjoint calls start from kernels.hpp's small-grid forward
// transform of the portraits).  User PSFs, vector, padded and batched plans keep the
// passes of kernels.hpp.
#pragma once
#include "kernels.hpp"

namespace mh3d {

// Intermediate layouts: cp[y0][x][column] (the plane pass's folded shares) and
// qx[x][column] (the column pass's output), so each plane workgroup reads and writes one
// contiguous run; the column pass takes its columns in runs of CPC.
//
// Plan-time tables of the separable passes (FP64 sums, FP32 storage):
//   sfs[k][qx]        scale_k F_k(qx) (its real part, or its imaginary part when bit k of
//                     imag_mask is set), the x factor of the stored spectra
//   set[y0][q'y][qz]  Et(y0, q'y, qz) = sum_jy w_ny^(y0 qy) Ehat(qy, qz), qz <= nz/2
__global__ void k_sep_tables(Geo g, const double2* __restrict__ fhat, const double2* __restrict__ ehat,
                             const double* __restrict__ scale, uint32_t imag_mask,
                             const double2* __restrict__ tw64y, float* __restrict__ sfs, float2* __restrict__ set) {
  const int nf = g.K * g.nx;
  const int ne = g.sy * g.my * g.nzh;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nf + ne; t += gridDim.x * blockDim.x) {
    if (t < nf) {
      const int k = t / g.nx;
      const double2 f = fhat[t];
      sfs[t] = (float)((((imag_mask >> k) & 1u) ? f.y : f.x) * scale[k]);
    } else {
      const int r = t - nf;
      const int y0 = r / (g.my * g.nzh), r2 = r - y0 * (g.my * g.nzh);
      const int qyp = r2 / g.nzh, qz = r2 - qyp * g.nzh;
      double sr = 0.0, si = 0.0;
      for (int jy = 0; jy < g.sy; ++jy) {
        const int qy = qyp + jy * g.my;
        const double2 w = tw64y[(long long)y0 * qy % g.ny];   // exp(-2 pi i y0 qy / ny)
        const double2 e = ehat[(long long)qy * g.nzh + qz];
        sr += w.x * e.x - w.y * e.y;
        si += w.x * e.y + w.y * e.x;
      }
      set[r] = make_float2((float)sr, (float)si);
    }
  }
}

template <int NX_, int NY_, int NZ_, int SX_, int SY_, int SZ_, int CPC_, int KMAX_, int TP_ = 256, int TPF_ = 256,
          int LSX_ = 0, int LSZ_ = 0>
struct FastGeo {
  static constexpr int NX = NX_, NY = NY_, NZ = NZ_, SX = SX_, SY = SY_, SZ = SZ_;
  static constexpr int MX = NX / SX, MY = NY / SY, MZ = NZ / SZ;
  static constexpr int NZH = NZ / 2 + 1, MZH = MZ / 2 + 1;
  static constexpr int NCLS = MY * MZH;                     // columns (q'y, q'z)
  static constexpr int CPC = CPC_, KMAX = KMAX_;
  static constexpr int TC = CPC * MX;                       // column-pass threads: one per (column, q'x)
  // line strides of the x lines (column pass) and packed z lines (plane passes): odd by
  // default; a geometry may set others where its line count per wave makes an odd stride
  // put several lanes of a stage on one bank (with 4 x lines per block a stride of 1 mod
  // 32 complex values does; 6 mod 32 spreads them)
  static constexpr int LSX = LSX_ ? LSX_ : (NX | 1), LSZ = LSZ_ ? LSZ_ : (NZ | 1), LSY = MY | 1;
  static constexpr int NP = MY / 2;                         // row pairs of a plane block
  static constexpr int TP = TP_;                            // adjoint plane-pass threads
  static constexpr int TPF = TPF_;                          // forward plane-pass threads
  static constexpr int NBP = NX * SY;                       // plane-pass blocks (x-plane, y0)
  // one plane-pass LDS buffer: packed row pairs or half-spectrum columns (+ the staged Q)
  static constexpr int PB0 = NP * LSZ, PB1 = NZH * LSY;
  static constexpr int PBUF = PB0 > PB1 ? PB0 : PB1;
  static constexpr size_t LDS_PLANE = sizeof(float2) * (NZ + MY + 2 * (size_t)PBUF + NCLS);
  static constexpr int LSM = MX | 1;                        // line stride of the column pass's x' lines
  static constexpr size_t LDS_COL = sizeof(float2) * (NX + MX + 2 * (size_t)CPC * LSX + 2 * (size_t)KMAX * CPC * LSM);
  // small-grid inverse pass: packed row pairs of xb x'-planes or half-spectrum columns
  static constexpr int LSMY = MY | 1, LSMZ = MZ | 1;
  static constexpr size_t small_lds(int xb) {
    const size_t a = (size_t)((xb * MY + 1) / 2) * LSMZ, b = (size_t)xb * MZH * LSMY;
    return sizeof(float2) * (MY + MZ + 2 * (a > b ? a : b));
  }
  static_assert(MY % 2 == 0, "row pairs: my must be even");
  static_assert(NZ % 4 == 0, "rows are loaded as float4");
  static_assert(MZ % 2 == 0, "the decimated z-axis is even");
  static_assert(NCLS % CPC == 0, "columns per block must divide the columns");
  static_assert(TC <= 1024, "column block too large");
};

// Stockham stages of NL lines of length N held at l*LS + p (LS odd) with consecutive
// lanes on consecutive lines (the same butterfly of each): with an odd line stride the
// strided stores of a stage fall in distinct banks, and the lanes of a butterfly
// position share its twiddles (one broadcast read).  ld(l, p) gives element p of line l.
template <int N, int R, int NS, int SGN, int NL, int LS, class Load>
__device__ __forceinline__ void lf_stage_ld(Load ld, float2* __restrict__ out, const float2* tw) {
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
  constexpr int total = NL * NB;
  for (int b = threadIdx.x; b < total; b += blockDim.x) {
    const int l = b % NL, j = b / NL;
    const int k = j % NS;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ld(l, j + r * NB);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const float2 w = tw[k * r * TWS];
        v[r] = SGN < 0 ? cmul(v[r], w) : cmulcj(w, v[r]);
      }
    }
    dft<R, SGN>(v);
    const int o = l * LS + (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[o + r * NS] = v[r];
  }
}

template <int N, int R, int NS, int SGN, int NL, int LS>
__device__ __forceinline__ void lf_stage(const float2* __restrict__ in, float2* __restrict__ out, const float2* tw) {
  lf_stage_ld<N, R, NS, SGN, NL, LS>([&](int l, int p) { return in[l * LS + p]; }, out, tw);
}

// Radix of stage s: length-128 lines in groups of at least 16 (the plane passes' packed
// z lines) take 16 then 8, one stage and one barrier fewer than 8, 8, 2 (with fewer
// lines the radix-16 stage leaves too many lanes idle); otherwise ct_radix.
__host__ __device__ constexpr int lf_radix(int n, int s, int nl) {
  if (n == 128 && nl >= 16) return s == 0 ? 16 : (s == 1 ? 8 : 0);
  return ct_radix(n, s);
}

// Length-N transforms (unnormalised) of NL lines in *a, ping-ponging with *b; a barrier
// ends each stage.  Returns the buffer holding the result.  No leading barrier.
template <int N, int S, int NS, int SGN, int NL, int LS>
__device__ __forceinline__ float2* lf_fft(float2* a, float2* b, const float2* tw) {
  constexpr int R = lf_radix(N, S, NL);
  if constexpr (R == 0) {
    return a;
  } else {
    lf_stage<N, R, NS, SGN, NL, LS>(a, b, tw);
    __syncthreads();
    return lf_fft<N, S + 1, NS * R, SGN, NL, LS>(b, a, tw);
  }
}

// The same with the first stage's inputs from ld (computed from another buffer, which
// the first stage is the last to read): the first stage writes *a, the rest ping-pong
// between *a and *b.
template <int N, int SGN, int NL, int LS, class Load>
__device__ __forceinline__ float2* lf_fft_ld(Load ld, float2* a, float2* b, const float2* tw) {
  constexpr int R = lf_radix(N, 0, NL);
  lf_stage_ld<N, R, 1, SGN, NL, LS>(ld, a, tw);
  __syncthreads();
  return lf_fft<N, 1, R, SGN, NL, LS>(a, b, tw);
}

// Plane-pass block b -> (x-plane, y0).  The blocks of one XCD (b mod 8) take a run of
// consecutive planes with all their y0, so the stencil's neighbouring planes and the
// column pass's runs of x share that XCD's L2.
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

// ============================================================================ plane pass (forward)
// Block (x, y0): u = b . a on rows y = sy*y1 + y0 of plane x (a: rho, y^k or s w by SRC),
// R2C along z, length-my DFT along y1, then the share C(y0; x, q'y, q'z) of the folded
// plane into cp[y0][x][column].
template <class G, int SRC>
__global__ __launch_bounds__(G::TPF) void k_fast_plane_fwd(const VolDesc* __restrict__ vds, const float* __restrict__ a) {
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
  const int t = threadIdx.x;
  // items (row pair j, 4 columns): rows 2j and 2j+1 of the block become the real and
  // imaginary parts of packed line j
  constexpr int F4R = G::NZ / 4, F4 = G::NP * F4R, NL = (F4 + G::TPF - 1) / G::TPF;
  const long long pb = (long long)x * G::NY * G::NZ;
  const float* __restrict__ bs = vd.b;
  float4 va[NL][2], vb[NL][2];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int f = t + G::TPF * i;
    if (f < F4) {
      const int j = f / F4R, c4 = f - (f / F4R) * F4R;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const long long off = pb + (long long)(G::SY * (2 * j + h) + y0) * G::NZ + 4 * c4;
        va[i][h] = ldg(reinterpret_cast<const float4*>(a + off));
        vb[i][h] = ldg(reinterpret_cast<const float4*>(bs + off));
      }
    }
  }
  // the table Et of this y0 for the block's output columns (SZ values per column)
  constexpr int NC = (G::NCLS + G::TPF - 1) / G::TPF;
  const float2* __restrict__ et = vd.set + (long long)y0 * G::MY * G::NZH;
  float2 ev[NC][G::SZ];
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    const int c = t + G::TPF * i;
    if (c < G::NCLS) {
      const int qyp = c / G::MZH, qzp = c - (c / G::MZH) * G::MZH;
#pragma unroll
      for (int jz = 0; jz < G::SZ; ++jz) {
        const int qz = qzp + G::MZ * jz;
        ev[i][jz] = ldg(et + qyp * G::NZH + (2 * qz <= G::NZ ? qz : G::NZ - qz));
      }
    }
  }
  load_table(twz, vd.tw + vd.off[2], G::NZ);
  load_table(twy, vd.tw + vd.off[4], G::MY);
  float c = 1.f;
  if constexpr (SRC == SRC_SCALED) c = (float)vd.st->scale;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int f = t + G::TPF * i;
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
      float2* d2 = B0 + j * G::LSZ + 4 * c4;
#pragma unroll
      for (int q = 0; q < 4; ++q) d2[q] = make_float2(u[0][q], u[1][q]);
    }
  }
  __syncthreads();
  float2* Z = lf_fft<G::NZ, 0, 1, -1, G::NP, G::LSZ>(B0, B1, twz);
  float2* X = (Z == B0) ? B1 : B0;
  // the y1 transform of the half-spectrum columns (line qz, element y1): its first stage
  // splits each packed pair into its two half spectra as it reads them
  auto split = [&](int q, int y1) {
    const int j = y1 >> 1;
    const float2 zq = Z[j * G::LSZ + q];
    const float2 zm = Z[j * G::LSZ + (q == 0 ? 0 : G::NZ - q)];
    return (y1 & 1) ? make_float2(0.5f * (zq.y + zm.y), -0.5f * (zq.x - zm.x))
                    : make_float2(0.5f * (zq.x + zm.x), 0.5f * (zq.y - zm.y));
  };
  const float2* Y = lf_fft_ld<G::MY, -1, G::NZH, G::LSY>(split, X, Z, twy);
  // this residue's share of the folded plane
  float2* __restrict__ dst = vd.cp + ((long long)y0 * G::NX + x) * G::NCLS;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    const int cc = t + G::TPF * i;
    if (cc < G::NCLS) {
      const int qyp = cc / G::MZH, qzp = cc - (cc / G::MZH) * G::MZH;
      float sx = 0.f, sy = 0.f;
#pragma unroll
      for (int jz = 0; jz < G::SZ; ++jz) {
        const int qz = qzp + G::MZ * jz;
        float2 v;
        if (2 * qz <= G::NZ) {
          v = Y[qz * G::LSY + qyp];
        } else {
          const float2 w = Y[(G::NZ - qz) * G::LSY + (qyp == 0 ? 0 : G::MY - qyp)];
          v = make_float2(w.x, -w.y);
        }
        const float2 e = ev[i][jz];
        sx += e.x * v.x - e.y * v.y;
        sy += e.x * v.y + e.y * v.x;
      }
      stg(dst + cc, make_float2(sx, sy));
    }
  }
}

// ============================================================================ column pass
// Modes beyond the fused ones (NRM_RESID, NRM_PLAIN, NRM_STORE of kernels.hpp): A alone
// (the forward products and G, no adjoint) and A^T alone (R_k from the small-grid spectra
// of the portraits that k_small_fwd left in G', no forward products).
enum { COL_FWD = 16, COL_ADJ = 17 };

// Column block of workgroup b: the workgroups of one XCD (b mod 8) take a run of
// consecutive column blocks, so the blocks that share a cache line of the shares, of
// G' and of Q read and write it through one L2.
template <class G>
__device__ __forceinline__ int fast_col_block(int b) {
  constexpr int NB = G::NCLS / G::CPC;
  if constexpr (NB % 8 == 0) return (b & 7) * (NB / 8) + (b >> 3);
  else return b;
}

// Block: CPC columns (q'y, q'z), one thread per (column, q'x) owning the x aliases
// qx = q'x + mx*jx.  Sums the sy shares of each column, transforms along x, then per
// harmonic Fhat_k(q'x) = sum_jx F_k(qx) W(qx) (times i for imaginary F_k), the residual
// R_k = M Fhat_k (- the data's spectrum D_k in NRM_RESID), and Q(qx) = sum_k conj(F_k(qx))
// R_k(q'x); Q transformed back along x goes to qx[x][column] for the adjoint plane
// pass.  NRM_STORE also writes the portraits' decimated spectra G (inverse x' transform
// of Fhat) for the small-grid pass; M Fhat then stands for the spectra of d itself.
//
// grid.y > 1 runs one descriptor per y-block (the back-projections of single harmonics).
template <class G, int MODE>
__global__ __launch_bounds__(G::TC) void k_fast_col(const VolDesc* __restrict__ vds, int check_done) {
  const VolDesc& vd = vds[blockIdx.y];
  if (check_done && vd.st->done) return;
  constexpr int NX = G::NX, MX = G::MX, SX = G::SX, CPC = G::CPC, KMAX = G::KMAX, LSX = G::LSX;
  constexpr bool kFwd = MODE != COL_ADJ, kAdj = MODE != COL_FWD;
  constexpr bool kStoreG = MODE == NRM_STORE || MODE == COL_FWD;
  const int c0 = fast_col_block<G>(blockIdx.x) * CPC;
  const int K = vd.g.K;
  extern __shared__ float2 lds[];
  float2* twx = lds;
  float2* twm = twx + NX;
  float2* U0 = twm + MX;
  float2* U1 = U0 + CPC * LSX;
  constexpr int LSM = G::LSM;
  float2* F0 = U1 + CPC * LSX;
  float2* F1 = F0 + KMAX * CPC * LSM;
  const int t = threadIdx.x;
  const int cl = t / MX, qxp = t - (t / MX) * MX;
  // the shares of the block's columns: consecutive threads take consecutive columns of one x
  constexpr int NIT = CPC * NX, NI = (NIT + G::TC - 1) / G::TC;
  float2 sv[NI][G::SY];
  if constexpr (kFwd) {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int it = t + i * G::TC;
      if (NIT % G::TC == 0 || it < NIT) {
        const int xx = it / CPC, c = it - (it / CPC) * CPC;
#pragma unroll
        for (int y0 = 0; y0 < G::SY; ++y0) sv[i][y0] = ldg(vd.cp + ((long long)y0 * NX + xx) * G::NCLS + c0 + c);
      }
    }
  }
  // A^T alone: the portraits' small-grid spectra G'[k][x'-block][column][x'-in-block]
  if constexpr (MODE == COL_ADJ) {
    const int xb = vd.g.xb, nxb = MX / xb;
    for (int p = t; p < K * CPC * MX; p += G::TC) {
      const int k = p / (CPC * MX), r = p - k * (CPC * MX);
      const int c = r / MX, qq = r - c * MX;
      const int xbi = qq / xb, xi = qq - xbi * xb;
      F0[(k * CPC + c) * LSM + qq] = ldg(vd.Gp + (((long long)k * nxb + xbi) * G::NCLS + c0 + c) * xb + xi);
    }
  }
  // x factors of the thread's aliases and (residual) the data's spectra
  float fs[KMAX][SX];
  float2 dt[MODE == NRM_RESID ? KMAX : 1];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
#pragma unroll
      for (int jx = 0; jx < SX; ++jx) fs[k][jx] = ldg(vd.sfs + k * NX + qxp + jx * MX);
      if constexpr (MODE == NRM_RESID) dt[k] = ldg(vd.Gp + ((long long)k * G::NCLS + c0 + cl) * MX + qxp);
    }
  }
  load_table(twx, vd.tw + vd.off[0], NX);
  load_table(twm, vd.tw + vd.off[3], MX);
  const uint32_t imag_mask = vd.imag_mask;
  float2 w[SX];
  if constexpr (kFwd) {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int it = t + i * G::TC;
      if (NIT % G::TC == 0 || it < NIT) {
        const int xx = it / CPC, c = it - (it / CPC) * CPC;
        float2 s = sv[i][0];
#pragma unroll
        for (int y0 = 1; y0 < G::SY; ++y0) s = cadd(s, sv[i][y0]);
        U0[c * LSX + xx] = s;
      }
    }
    __syncthreads();
    float2* U = lf_fft<NX, 0, 1, -1, CPC, LSX>(U0, U1, twx);
#pragma unroll
    for (int jx = 0; jx < SX; ++jx) w[jx] = U[cl * LSX + qxp + jx * MX];
  }
  const float2* Rt = nullptr;   // A^T alone: R_k(q'x) = x' transform of the portraits' spectra
  if constexpr (MODE == COL_ADJ) {
    __syncthreads();
    Rt = lf_fft<MX, 0, 1, -1, KMAX * CPC, LSM>(F0, F1, twm);
  }
  const float Mf = (float)(G::MX * G::MY * G::MZ);
  float2 q[SX];
#pragma unroll
  for (int jx = 0; jx < SX; ++jx) q[jx] = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      const bool im = (imag_mask >> k) & 1u;
      float2 R;
      if constexpr (kFwd) {
        float fx = 0.f, fy = 0.f;
#pragma unroll
        for (int jx = 0; jx < SX; ++jx) { fx += fs[k][jx] * w[jx].x; fy += fs[k][jx] * w[jx].y; }
        const float2 f = im ? make_float2(-fy, fx) : make_float2(fx, fy);
        if constexpr (kStoreG) F0[(k * CPC + cl) * LSM + qxp] = f;
        R = make_float2(Mf * f.x, Mf * f.y);
        if constexpr (MODE == NRM_RESID) R = csub(R, dt[k]);
      } else {
        R = Rt[(k * CPC + cl) * LSM + qxp];
      }
      if constexpr (kAdj) {
        if (im) R = make_float2(R.y, -R.x);   // conj(i F) R = -i F R
#pragma unroll
        for (int jx = 0; jx < SX; ++jx) { q[jx].x += fs[k][jx] * R.x; q[jx].y += fs[k][jx] * R.y; }
      }
    }
  }
  if constexpr (kAdj) {
    __syncthreads();   // every thread has read its aliases of U
#pragma unroll
    for (int jx = 0; jx < SX; ++jx) U0[cl * LSX + qxp + jx * MX] = q[jx];
    __syncthreads();
    const float2* V = lf_fft<NX, 0, 1, +1, CPC, LSX>(U0, U1, twx);
    for (int it = t; it < NIT; it += G::TC) {
      const int xx = it / CPC, c = it - (it / CPC) * CPC;
      stg(vd.qx + (long long)xx * G::NCLS + c0 + c, V[c * LSX + xx]);
    }
  }
  if constexpr (kStoreG) {
    __syncthreads();
    const float2* F = lf_fft<MX, 0, 1, +1, KMAX * CPC, LSM>(F0, F1, twm);
    float2* __restrict__ Gs = vd.G;
    const int xb = vd.g.xb, nxb = MX / xb;
    for (int p = t; p < K * CPC * MX; p += G::TC) {
      const int k = p / (CPC * MX), r = p - k * (CPC * MX);
      const int xbi = r / (CPC * xb), r2 = r - xbi * (CPC * xb);
      const int c = r2 / xb, xi = r2 - c * xb;
      stg(Gs + (((long long)k * nxb + xbi) * G::NCLS + c0 + c) * xb + xi, F[(k * CPC + c) * LSM + xbi * xb + xi]);
    }
  }
}

// ============================================================================ solver step
// The end of a solver step on the block's voxels (rows y = sy*y1 + y0 of plane x), with
// u = b . v from the packed rows Z in LDS: the same arithmetic as StepCtx (kernels.hpp),
//   UPD_NORMAL  out = u + lam R(s w);  FP64 <s w, out>, ||out||^2
//   UPD_FISTA   g = u + lam R(y^k); rho^{k+1} = max(y^k - tau g, 0);
//               y^{k+1} = rho^{k+1} + k/(k+3) (rho^{k+1} - rho^k); FP64 ||rho^{k+1} - y^k||^2,
//               ||rho^{k+1}||^2, count of non-finite g
// with R the periodic 13-point stencil of stacked second differences (T = I for
// reg_kind 1) plus alpha on the boundary shell.  Items are 4 consecutive voxels along z:
// the point and its y and x neighbours are float4 loads, the z neighbours two more on
// each side.  FP64 block partials go to vd.partials[lb] (k_vol_finish sums them).
template <class G, int UPD>
__device__ __forceinline__ void fast_step(const VolDesc& vd, const AdjOut& ao, const float2* __restrict__ Z, int x, int y0,
                                          int lb) {
  constexpr int NV = UPD == UPD_NORMAL ? 2 : 3;
  constexpr int F4R = G::NZ / 4, NIT = G::MY * F4R;
  constexpr long long PL = (long long)G::NY * G::NZ;
  __shared__ double red[64];
  const DevState* st = vd.st;
  const int kk = st->k;
  const float* __restrict__ yv = (UPD == UPD_NORMAL) ? (ao.yin ? ao.yin : vd.rho[kk & 1]) : vd.y[kk & 1];
  const float* __restrict__ rk = vd.rho[kk & 1];
  float* __restrict__ out = (UPD == UPD_NORMAL) ? (ao.out ? ao.out : vd.rho[(kk + 1) & 1]) : nullptr;
  float* __restrict__ rho_next = vd.rho[(kk + 1) & 1];
  float* __restrict__ y_next = vd.y[(kk + 1) & 1];
  const float s = (UPD == UPD_NORMAL) ? (float)st->scale : 1.f;
  const float lam = vd.lam, alpha = vd.alpha, tau = (float)st->tau;
  const float beta1 = (float)((double)kk / (kk + 3.0));
  const bool stencil = vd.reg_kind == 0;
  const int aw = vd.aw;
  const float* __restrict__ bs = vd.b;
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  auto ld4 = [](const float* p) { return ldg(reinterpret_cast<const float4*>(p)); };
  auto wrap = [](int q, int n) { return q < 0 ? q + n : (q >= n ? q - n : q); };
  constexpr int U = 2;   // items whose loads are in flight together
  for (int f0 = threadIdx.x; f0 < NIT; f0 += U * G::TP) {
    float4 c[U], ym2[U], ym1[U], yp1[U], yp2[U], xm2[U], xm1[U], xp1[U], xp2[U], rv[U], bv[U];
    float zl2[U], zl1[U], zr1[U], zr2[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int f = f0 + q * G::TP;
      if (f >= NIT) break;
      const int y1 = f / F4R, z0 = 4 * (f - (f / F4R) * F4R);
      const int y = G::SY * y1 + y0;
      const long long row = (long long)x * PL + (long long)y * G::NZ;
      const long long i0 = row + z0;
      c[q] = ld4(yv + i0);
      bv[q] = ld4(bs + i0);
      if (UPD == UPD_FISTA) rv[q] = ld4(rk + i0);
      if (stencil) {
        zl2[q] = ldg(yv + row + wrap(z0 - 2, G::NZ));
        zl1[q] = ldg(yv + row + wrap(z0 - 1, G::NZ));
        zr1[q] = ldg(yv + row + wrap(z0 + 4, G::NZ));
        zr2[q] = ldg(yv + row + wrap(z0 + 5, G::NZ));
        const long long pln = (long long)x * PL + z0;
        ym2[q] = ld4(yv + pln + (long long)wrap(y - 2, G::NY) * G::NZ);
        ym1[q] = ld4(yv + pln + (long long)wrap(y - 1, G::NY) * G::NZ);
        yp1[q] = ld4(yv + pln + (long long)wrap(y + 1, G::NY) * G::NZ);
        yp2[q] = ld4(yv + pln + (long long)wrap(y + 2, G::NY) * G::NZ);
        const long long col = (long long)y * G::NZ + z0;
        xm2[q] = ld4(yv + (long long)wrap(x - 2, G::NX) * PL + col);
        xm1[q] = ld4(yv + (long long)wrap(x - 1, G::NX) * PL + col);
        xp1[q] = ld4(yv + (long long)wrap(x + 1, G::NX) * PL + col);
        xp2[q] = ld4(yv + (long long)wrap(x + 2, G::NX) * PL + col);
      }
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int f = f0 + q * G::TP;
      if (f >= NIT) break;
      const int y1 = f / F4R, z0 = 4 * (f - (f / F4R) * F4R);
      const int y = G::SY * y1 + y0;
      const long long i0 = (long long)x * PL + (long long)y * G::NZ + z0;
      const float2* zr = Z + (y1 >> 1) * G::LSZ + z0;
      const float cv[4] = {c[q].x, c[q].y, c[q].z, c[q].w};
      const float zrow[8] = {zl2[q], zl1[q], c[q].x, c[q].y, c[q].z, c[q].w, zr1[q], zr2[q]};
      const float a_ym2[4] = {ym2[q].x, ym2[q].y, ym2[q].z, ym2[q].w}, a_ym1[4] = {ym1[q].x, ym1[q].y, ym1[q].z, ym1[q].w};
      const float a_yp1[4] = {yp1[q].x, yp1[q].y, yp1[q].z, yp1[q].w}, a_yp2[4] = {yp2[q].x, yp2[q].y, yp2[q].z, yp2[q].w};
      const float a_xm2[4] = {xm2[q].x, xm2[q].y, xm2[q].z, xm2[q].w}, a_xm1[4] = {xm1[q].x, xm1[q].y, xm1[q].z, xm1[q].w};
      const float a_xp1[4] = {xp1[q].x, xp1[q].y, xp1[q].z, xp1[q].w}, a_xp2[4] = {xp2[q].x, xp2[q].y, xp2[q].z, xp2[q].w};
      const float a_b[4] = {bv[q].x, bv[q].y, bv[q].z, bv[q].w};
      const float a_r[4] = {rv[q].x, rv[q].y, rv[q].z, rv[q].w};
      float o4[4], n4[4], m4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma clang fp contract(off)
        const int z = z0 + e;
        const float vz = (y1 & 1) ? zr[e].y : zr[e].x;
        const float u = __fmul_rn(a_b[e], vz);
        float t;
        if (!stencil) {
          t = s * cv[e];
        } else {
          t = 18.f * (s * cv[e]);
          t += s * (zrow[e + 4] + zrow[e]) - 4.f * s * (zrow[e + 3] + zrow[e + 1]);
          t += s * (a_yp2[e] + a_ym2[e]) - 4.f * s * (a_yp1[e] + a_ym1[e]);
          t += s * (a_xp2[e] + a_xm2[e]) - 4.f * s * (a_xp1[e] + a_xm1[e]);
        }
        if (alpha > 0.f) {
          const bool shell = x < aw || x >= G::NX - aw || y < aw || y >= G::NY - aw || z < aw || z >= G::NZ - aw;
          if (shell) t += alpha * (s * cv[e]);
        }
        if constexpr (UPD == UPD_NORMAL) {
          const float o = u + lam * t;
          o4[e] = o;
          acc[0] += (double)(s * cv[e]) * (double)o;
          acc[1] += (double)o * (double)o;
        } else {
          const float yk = cv[e];
          const float gr = u + lam * t;
          const float rn = fmaxf(yk - tau * gr, 0.f);
          n4[e] = rn;
          m4[e] = rn + beta1 * (rn - a_r[e]);
          const double dd = (double)rn - (double)yk;
          acc[0] += dd * dd;
          acc[1] += (double)rn * (double)rn;
          if (!isfinite(gr) || !isfinite(yk)) acc[2] += 1.0;
        }
      }
      if constexpr (UPD == UPD_NORMAL) {
        stg(reinterpret_cast<float4*>(out + i0), make_float4(o4[0], o4[1], o4[2], o4[3]));
      } else {
        stg(reinterpret_cast<float4*>(rho_next + i0), make_float4(n4[0], n4[1], n4[2], n4[3]));
        stg(reinterpret_cast<float4*>(y_next + i0), make_float4(m4[0], m4[1], m4[2], m4[3]));
      }
    }
  }
  store_step_partials<NV>(vd, acc, red, lb);
}

// ============================================================================ plane pass (adjoint)
// Block (x, y0): the residue's half spectrum Q(x, q'y, qz mod mz) conj(Et(y0, q'y, qz)),
// inverse length-my DFT along y1, C2R along z, then per voxel of rows y = sy*y1 + y0:
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
  float2* Qs = B1 + G::PBUF;   // Q(x, column)
  const int t = threadIdx.x;
  const long long pb = (long long)x * G::NY * G::NZ;
  const float* __restrict__ bs = vd.b;
  // every load is issued before the first is used: Q of the plane, the table Et of y0
  // and, for A^T, the sensitivity rows of the output
  constexpr int NQ = (G::NCLS + G::TP - 1) / G::TP;
  float2 qv[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int c = t + i * G::TP;
    if (c < G::NCLS) qv[i] = ldg(vd.qx + (long long)x * G::NCLS + c);
  }
  constexpr int NE = G::NZH * G::MY, NEI = (NE + G::TP - 1) / G::TP;
  const float2* __restrict__ et = vd.set + (long long)y0 * G::MY * G::NZH;
  float2 ev[NEI];
#pragma unroll
  for (int i = 0; i < NEI; ++i) {
    const int it = t + i * G::TP;
    if (it < NE) ev[i] = ldg(et + it);   // [q'y][qz]
  }
  constexpr int F4R = G::NZ / 4, P4 = G::NP * F4R, NB4 = (P4 + G::TP - 1) / G::TP;
  float4 bq[kStep ? 1 : NB4][2];
  if constexpr (!kStep) {
#pragma unroll
    for (int i = 0; i < NB4; ++i) {
      const int f = t + i * G::TP;
      if (f < P4) {
        const int j = f / F4R, c4 = f - (f / F4R) * F4R;
        const long long o0 = pb + (long long)(G::SY * 2 * j + y0) * G::NZ + 4 * c4;
        bq[i][0] = ldg(reinterpret_cast<const float4*>(bs + o0));
        bq[i][1] = ldg(reinterpret_cast<const float4*>(bs + o0 + (long long)G::SY * G::NZ));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int c = t + i * G::TP;
    if (c < G::NCLS) Qs[c] = qv[i];
  }
  load_table(twz, vd.tw + vd.off[2], G::NZ);
  load_table(twy, vd.tw + vd.off[4], G::MY);
  __syncthreads();
  // half spectrum, columns B0[qz][q'y]
#pragma unroll
  for (int i = 0; i < NEI; ++i) {
    const int it = t + i * G::TP;
    if (it < NE) {
      const int qyp = it / G::NZH, qz = it - (it / G::NZH) * G::NZH;
      const int qzr = qz % G::MZ;
      float2 qq;
      if (2 * qzr <= G::MZ) {
        qq = Qs[qyp * G::MZH + qzr];
      } else {   // Q is Hermitian over (q'y, q'z)
        const float2 w = Qs[(qyp == 0 ? 0 : G::MY - qyp) * G::MZH + (G::MZ - qzr)];
        qq = make_float2(w.x, -w.y);
      }
      B0[qz * G::LSY + qyp] = cmulcj(ev[i], qq);   // conj(Et) Q
    }
  }
  __syncthreads();
  float2* X = lf_fft<G::MY, 0, 1, +1, G::NZH, G::LSY>(B0, B1, twy);
  float2* Zb = (X == B0) ? B1 : B0;
  // C2R along z of the packed rows Z[j] = X[2j] + i X[2j+1] (Hermitian extension for
  // qz > nz/2): the first stage of the z transform packs its inputs as it reads them
  auto pack = [&](int j, int q) {
    const bool upper = 2 * q > G::NZ;
    const int qq = upper ? G::NZ - q : q;
    float2 xv = X[qq * G::LSY + 2 * j];
    float2 yv = X[qq * G::LSY + 2 * j + 1];
    if (qq == 0 || 2 * qq == G::NZ) { xv.y = 0.f; yv.y = 0.f; }
    if (upper) { xv.y = -xv.y; yv.y = -yv.y; }
    return make_float2(xv.x - yv.y, xv.y + yv.x);
  };
  const float2* Z = lf_fft_ld<G::NZ, +1, G::NP, G::LSZ>(pack, Zb, X, twz);
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
      stg(reinterpret_cast<float4*>(out + o0), make_float4(b0.x * z0.x, b0.y * z1.x, b0.z * z2.x, b0.w * z3.x));
      stg(reinterpret_cast<float4*>(out + o1), make_float4(b1.x * z0.y, b1.y * z1.y, b1.z * z2.y, b1.w * z3.y));
    }
  } else {
    fast_step<G, OUT == OUT_STEP_NORMAL ? UPD_NORMAL : UPD_FISTA>(vd, ao, Z, x, y0, lb);
  }
}

// grid.y > 1 (OUT_SCALE_B only): descriptor y and output volume y of consecutive volumes.
template <class G, int OUT>
__global__ __launch_bounds__(G::TP) void k_fast_plane_adj(const VolDesc* __restrict__ vds, AdjOut ao) {
  if constexpr (OUT == OUT_SCALE_B) ao.out += (long long)blockIdx.y * G::NX * G::NY * G::NZ;
  fast_plane_adj_body<G, OUT>(vds[blockIdx.y], blockIdx.x, ao);
}

// ============================================================================ small-grid inverse
// Block (k, x'-block of XB planes): the portraits d_k of those planes from their decimated
// spectra G[k][x'-block][column][x'-in-block] (the column pass's output): inverse
// length-my transform along y', C2R along z' (row pairs packed), store.  The same
// transforms as small_inv_body<EPI_STORE> (kernels.hpp) on compile-time sizes.
template <class G, int XB>
__device__ __forceinline__ void fast_small_inv_body(const VolDesc& vd, int lb, float* __restrict__ d) {
  constexpr int MY = G::MY, MZ = G::MZ, MZH = G::MZH, LSMY = G::LSMY, LSMZ = G::LSMZ;
  constexpr int ROWS = XB * MY, NPR = (ROWS + 1) / 2, NXB = G::MX / XB;
  constexpr size_t A0 = (size_t)NPR * LSMZ, A1 = (size_t)XB * MZH * LSMY;
  constexpr int SB = A0 > A1 ? (int)A0 : (int)A1;
  extern __shared__ float2 lds[];
  float2* twy = lds;
  float2* twz = twy + MY;
  float2* P0 = twz + MZ;
  float2* P1 = P0 + SB;
  const int t = threadIdx.x, nt = blockDim.x;
  const int k = lb / NXB, xbi = lb - (lb / NXB) * NXB;
  const float2* __restrict__ src = vd.G + ((long long)k * NXB + xbi) * G::NCLS * XB;
  constexpr int NS = G::NCLS * XB;
  for (int p = t; p < NS; p += nt) {
    const float2 v = ldg(src + p);
    const int c = p / XB, xi = p - (p / XB) * XB;
    const int qyp = c / MZH, qzp = c - (c / MZH) * MZH;
    P0[(xi * MZH + qzp) * LSMY + qyp] = v;
  }
  load_table(twy, vd.tw + vd.off[4], MY);
  load_table(twz, vd.tw + vd.off[5], MZ);
  __syncthreads();
  float2* X = lf_fft<MY, 0, 1, +1, XB * MZH, LSMY>(P0, P1, twy);
  float2* Zb = (X == P0) ? P1 : P0;
  // C2R along z': row r = xi my + y', pairs (2j, 2j+1) packed by the first stage of the
  // z' transform as it reads them
  auto pack = [&](int j, int q) {
    const bool upper = 2 * q > MZ;
    const int qq = upper ? MZ - q : q;
    const int r0 = 2 * j, r1 = 2 * j + 1;
    float2 xv = X[((r0 / MY) * MZH + qq) * LSMY + r0 % MY];
    float2 yv = r1 < ROWS ? X[((r1 / MY) * MZH + qq) * LSMY + r1 % MY] : make_float2(0.f, 0.f);
    if (qq == 0 || 2 * qq == MZ) { xv.y = 0.f; yv.y = 0.f; }
    if (upper) { xv.y = -xv.y; yv.y = -yv.y; }
    return make_float2(xv.x - yv.y, xv.y + yv.x);
  };
  const float2* Z = lf_fft_ld<MZ, +1, NPR, LSMZ>(pack, Zb, X, twz);
  // store the block's rows: d[k][xbi XB + xi][y'][z'] is one contiguous run
  float* __restrict__ dst = d + (long long)k * G::MX * MY * MZ + (long long)xbi * XB * MY * MZ;
  constexpr int Q4 = ROWS * MZ / 4;
  for (int f = t; f < Q4; f += nt) {
    const int r = f / (MZ / 4), z4 = 4 * (f - (f / (MZ / 4)) * (MZ / 4));
    const float2* zr = Z + (r >> 1) * LSMZ + z4;
    float v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (r & 1) ? zr[e].y : zr[e].x;
    stg(reinterpret_cast<float4*>(dst + (long long)r * MZ + z4), make_float4(v[0], v[1], v[2], v[3]));
  }
}

template <class G>
__device__ __forceinline__ void fast_small_inv_dispatch(const VolDesc& vd, int lb, float* __restrict__ d) {
  switch (vd.g.xb) {
    case 1: fast_small_inv_body<G, 1>(vd, lb, d); break;
    case 2: fast_small_inv_body<G, 2>(vd, lb, d); break;
    case 4: fast_small_inv_body<G, 4>(vd, lb, d); break;
    default: fast_small_inv_body<G, 8>(vd, lb, d); break;
  }
}

template <class G>
__global__ __launch_bounds__(G::TP) void k_fast_small_inv(const VolDesc* __restrict__ vds, float* __restrict__ d) {
  fast_small_inv_dispatch<G>(vds[0], blockIdx.x, d);
}

// ============================================================================ small-grid forward
// Block (k, x'-block of XB planes): the small-grid spectra of the portraits r of those
// planes (A^T alone and the back-projections start here), written as k_small_fwd writes
// them, G'[k][x'-block][column][x'-in-block]: rows packed in pairs, R2C along z' (the
// pairs split into their half spectra by the first stage of the y' transform), the
// length-my transform along y'.
template <class G, int XB>
__device__ __forceinline__ void fast_small_fwd_body(const VolDesc& vd, int lb, const float* __restrict__ r,
                                                    float2* __restrict__ out) {
  constexpr int MY = G::MY, MZ = G::MZ, MZH = G::MZH, LSMY = G::LSMY, LSMZ = G::LSMZ;
  constexpr int ROWS = XB * MY, NPR = ROWS / 2, NXB = G::MX / XB;
  constexpr size_t A0 = (size_t)NPR * LSMZ, A1 = (size_t)XB * MZH * LSMY;
  constexpr int SB = A0 > A1 ? (int)A0 : (int)A1;
  extern __shared__ float2 lds[];
  float2* twy = lds;
  float2* twz = twy + MY;
  float2* P0 = twz + MZ;
  float2* P1 = P0 + SB;
  const int t = threadIdx.x, nt = blockDim.x;
  const int k = lb / NXB, xbi = lb - (lb / NXB) * NXB;
  // the block's rows (xi my + y') are one contiguous run of the portraits
  const float* __restrict__ src = r + (long long)k * G::MX * MY * MZ + (long long)xbi * XB * MY * MZ;
  constexpr int Q4 = ROWS * MZ / 4;
  float* Pf = reinterpret_cast<float*>(P0);
  for (int f = t; f < Q4; f += nt) {
    const int rr = f / (MZ / 4), z4 = 4 * (f - (f / (MZ / 4)) * (MZ / 4));
    const float4 v = ldg(reinterpret_cast<const float4*>(src + (long long)rr * MZ + z4));
    float* dst = Pf + 2 * ((rr >> 1) * LSMZ + z4) + (rr & 1);
    dst[0] = v.x; dst[2] = v.y; dst[4] = v.z; dst[6] = v.w;
  }
  load_table(twy, vd.tw + vd.off[4], MY);
  load_table(twz, vd.tw + vd.off[5], MZ);
  __syncthreads();
  float2* Z = lf_fft<MZ, 0, 1, -1, NPR, LSMZ>(P0, P1, twz);
  float2* X = (Z == P0) ? P1 : P0;
  // line (xi, q'z), element y': row xi my + y' of the packed pair (its real or imaginary half)
  auto split = [&](int l, int yp) {
    const int xi = l / MZH, q = l - (l / MZH) * MZH;
    const int rr = xi * MY + yp, j = rr >> 1;
    const float2 zq = Z[j * LSMZ + q];
    const float2 zm = Z[j * LSMZ + (q == 0 ? 0 : MZ - q)];
    return (rr & 1) ? make_float2(0.5f * (zq.y + zm.y), -0.5f * (zq.x - zm.x))
                    : make_float2(0.5f * (zq.x + zm.x), 0.5f * (zq.y - zm.y));
  };
  const float2* Y = lf_fft_ld<MY, -1, XB * MZH, LSMY>(split, X, Z, twy);
  float2* __restrict__ dst = out + ((long long)k * NXB + xbi) * G::NCLS * XB;
  for (int p = t; p < G::NCLS * XB; p += nt) {
    const int c = p / XB, xi = p - (p / XB) * XB;
    const int qyp = c / MZH, qzp = c - (c / MZH) * MZH;
    stg(dst + p, Y[(xi * MZH + qzp) * LSMY + qyp]);
  }
}

template <class G>
__global__ __launch_bounds__(G::TP) void k_fast_small_fwd(const VolDesc* __restrict__ vds, const float* __restrict__ r,
                                                        float2* __restrict__ out) {
  const VolDesc& vd = vds[0];
  switch (vd.g.xb) {
    case 1: fast_small_fwd_body<G, 1>(vd, blockIdx.x, r, out); break;
    case 2: fast_small_fwd_body<G, 2>(vd, blockIdx.x, r, out); break;
    case 4: fast_small_fwd_body<G, 4>(vd, blockIdx.x, r, out); break;
    default: fast_small_fwd_body<G, 8>(vd, blockIdx.x, r, out); break;
  }
}

// A then A^T after k_fast_col<NRM_STORE>: blocks [0, NBP) run the adjoint plane pass
// (ao.out = b . v), the others the small-grid inverse pass that writes the portraits d.
template <class G>
__global__ __launch_bounds__(G::TP) void k_fast_adj_and_store(const VolDesc* __restrict__ vds, AdjOut ao,
                                                            float* __restrict__ d) {
  const VolDesc& vd = vds[0];
  if ((int)blockIdx.x < G::NBP) fast_plane_adj_body<G, OUT_SCALE_B>(vd, blockIdx.x, ao);
  else fast_small_inv_dispatch<G>(vd, blockIdx.x - G::NBP, d);
}

}  // namespace mh3d
