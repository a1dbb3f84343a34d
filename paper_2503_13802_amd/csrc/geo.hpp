// Geometry of one MH3D plan, shared by host launch code and kernels.
//
// Spectra use an "alias-class" layout.  The decimated grid (mx, my, mz) has a
// Hermitian half along z, q'z in [0, mz/2].  A class is one pair (q'y, q'z),
// class id c = q'y * mzh + q'z, mzh = mz/2 + 1.  Its nmem = sy*sz members are the
// full-grid (qy, qz) = (q'y + jy*my, q'z + jz*mz), member id m = jy*sz + jz.  Folding
// the full spectrum onto the decimated grid (the Fourier form of the row selector
// P) sums exactly over the members of one class and over qx = q'x + jx*mx, so one
// workgroup can own a class end to end.  Members with qz > nz/2 are stored as the
// conjugate of the in-plane Hermitian partner (ny - qy, nz - qz), which is exact for
// the y-z spectrum of a real x-plane.
#pragma once
#include <stdint.h>

namespace mh3d {

// Division by a per-plan constant d >= 1 for 0 <= n < 2^31 with one 32x64-bit
// multiply: q = (n * m) >> s, m = ceil(2^(31+l) / d), l = ceil(log2 d)
// (Granlund & Montgomery, PLDI 1994, round-up variant).
struct FastDiv {
  uint64_t m;
  uint32_t s, d;
  __host__ __device__ inline uint32_t div(uint32_t n) const { return (uint32_t)(((uint64_t)n * m) >> s); }
  __host__ __device__ inline uint32_t mod(uint32_t n) const { return n - div(n) * d; }
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.d = d;
  f.s = 31 + l;
  const unsigned __int128 one = 1;
  const unsigned __int128 p = one << (31 + l);
  f.m = (uint64_t)((p + d - 1) / d);
  return f;
}

struct Geo {
  int nx, ny, nz, nzh;     // grid, nzh = nz/2 + 1
  int mx, my, mz, mzh;     // decimated grid, mzh = mz/2 + 1
  int sx, sy, sz, S;       // decimation factors, S = sx*sy*sz
  int nmem;                // members per class = sy*sz
  int ncls;                // classes = my*mzh
  int plane;               // complex values per x-plane of the class layout = ncls*nmem
  int K;                   // harmonics
  int C;                   // components of the vector model (1: scalar b and h_k)
  int cpw;                 // classes per class-kernel workgroup (divides ncls)
  int E;                   // spectrum elements per thread in the class kernel (divides S)
  int xb;                  // x' planes per small-grid workgroup (divides mx)
  int ps;                  // workgroups per x-plane in the plane passes (1 to 4)
  int npairs;              // (ny + 1)/2 row pairs of one full x-plane
  int spairs;              // (xb*my + 1)/2 row pairs of one small-grid workgroup
  int lsy;                 // LDS line stride of y-transforms in the plane kernels (ny + pad)
  int lsx;                 // LDS line stride of x-transforms in the class kernels (nx + pad)
  int lsmy;                // LDS line stride of y'-transforms in the small kernels (my + pad)
  long long N, M;          // nx*ny*nz, mx*my*mz
  int padded;              // boundary padding: the portraits cover only the field of view
  int pxs, pys, pzs;       // field-of-view offsets in decimated samples (padding / decimation)
  int mxf, myf, mzf;       // field-of-view portrait dims
  long long Mf;            // mxf*myf*mzf (= M without padding)
  long long hsz;           // spectrum elements per harmonic = ncls*mx*S = plane*nx
  FastDiv f_nz, f_nzh, f_nmem, f_mzh, f_sz, f_mz, f_W, f_xb, f_S, f_mxS, f_cpwmx, f_cpwxb, f_ny, f_my;
};

}  // namespace mh3d
