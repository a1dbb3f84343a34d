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

namespace mh3d {

struct Geo {
  int nx, ny, nz, nzh;     // grid, nzh = nz/2 + 1
  int mx, my, mz, mzh;     // decimated grid, mzh = mz/2 + 1
  int sx, sy, sz, S;       // decimation factors, S = sx*sy*sz
  int nmem;                // members per class = sy*sz
  int ncls;                // classes = my*mzh
  int plane;               // complex values per x-plane of the class layout = ncls*nmem
  int K;                   // harmonics
  int cpw;                 // classes per class-kernel workgroup (divides ncls)
  int E;                   // spectrum elements per thread in the class kernel (divides S)
  int xb;                  // x' planes per small-grid workgroup (divides mx)
  int npairs;              // (ny + 1)/2 row pairs of one full x-plane
  int spairs;              // (xb*my + 1)/2 row pairs of one small-grid workgroup
  long long N, M;          // nx*ny*nz, mx*my*mz
  long long hsz;           // spectrum elements per harmonic = ncls*mx*S = plane*nx
};

}  // namespace mh3d
