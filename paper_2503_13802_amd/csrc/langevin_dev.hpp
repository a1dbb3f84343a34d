// FP64 device evaluation of derivatives of the Langevin function
// L(u) = coth(u) - 1/u (paper Sec. 2), used at plan time to sample the PSFs of
// Sec. 3.3 eq. hkapprox.
//
// L is meromorphic with simple poles at u = i m pi (m != 0), each of residue 1
// (the analytic structure App. E uses for Prop. 2), so
//   L(u) = sum_{m>=1} [ 1/(u - i m pi) + 1/(u + i m pi) ],
//   L^(n)(u) = 2 (-1)^n n! sum_{m>=1} Re (u - i m pi)^{-(n+1)},   n >= 1.
// The series is summed directly for m < MD and the remainder sum_{m>=MD} g(m),
// g(x) = (u - i pi x)^{-q}, q = n + 1, by the Euler-Maclaurin formula
//   int_MD^inf g + g(MD)/2 - sum_p B_{2p}/(2p)! g^{(2p-1)}(MD),
// with g^{(r)}(x) = (i pi)^r q (q+1) ... (q+r-1) (u - i pi x)^{-q-r} and
// int_MD^inf g = -(u - i pi MD)^{1-q} / (i pi (q-1)).
#pragma once
#include <hip/hip_runtime.h>

namespace mh3d {

struct zc { double re, im; };
__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ zc zinv(zc a) {
  double s = 1.0 / (a.re * a.re + a.im * a.im);
  return {a.re * s, -a.im * s};
}
__device__ __forceinline__ zc zpow(zc a, int e) {  // e >= 0, by squaring
  zc r = {1.0, 0.0};
  while (e) {
    if (e & 1) r = zmul(r, a);
    a = zmul(a, a);
    e >>= 1;
  }
  return r;
}

// n >= 1.  Accurate to a few ulp-scale relative errors for all real u.
__device__ inline double langevin_deriv_dev(int n, double u) {
  const double PI = 3.14159265358979323846;
  const int MD = 40;
  // B_{2p} / (2p)!  for p = 1..8  (Bernoulli numbers 1/6, -1/30, 1/42, -1/30, 5/66,
  // -691/2730, 7/6, -3617/510 divided by 2!, 4!, ..., 16!)
  const double bc[8] = {
      1.0 / 6.0 / 2.0,
      -1.0 / 30.0 / 24.0,
      1.0 / 42.0 / 720.0,
      -1.0 / 30.0 / 40320.0,
      5.0 / 66.0 / 3628800.0,
      -691.0 / 2730.0 / 479001600.0,
      7.0 / 6.0 / 87178291200.0,
      -3617.0 / 510.0 / 20922789888000.0};
  const int q = n + 1;
  zc acc = {0.0, 0.0};
  for (int m = MD - 1; m >= 1; --m) {
    zc w = zinv(zc{u, -PI * m});
    zc t = zpow(w, q);
    acc.re += t.re;
    acc.im += t.im;
  }
  zc inv = zinv(zc{u, -PI * MD});          // 1/(u - i pi MD)
  zc invq1 = zpow(inv, q - 1);             // (u - i pi MD)^{1-q}
  zc invq = zmul(invq1, inv);              // (u - i pi MD)^{-q}
  // -(w^{1-q}) / (i pi (q-1)):  1/i = -i  ->  -(a)(-i)/(pi(q-1)) = i a / (pi (q-1))
  double c = 1.0 / (PI * (q - 1));
  zc tail = {-invq1.im * c, invq1.re * c};
  tail.re += 0.5 * invq.re;
  tail.im += 0.5 * invq.im;
  zc ipi = {0.0, PI};
  zc pw = invq;                            // w^{-q-r}, starting r = 0
  zc ipr = {1.0, 0.0};                     // (i pi)^r
  double rising = 1.0;                     // q (q+1) ... (q+r-1)
  int r = 0;
  for (int p = 1; p <= 8; ++p) {
    const int rt = 2 * p - 1;
    while (r < rt) {
      rising *= (double)(q + r);
      pw = zmul(pw, inv);
      ipr = zmul(ipr, ipi);
      ++r;
    }
    zc d = zmul(ipr, pw);
    tail.re -= bc[p - 1] * rising * d.re;
    tail.im -= bc[p - 1] * rising * d.im;
  }
  double fact = 1.0;
  for (int t = 2; t <= n; ++t) fact *= (double)t;
  const double sgn = (n & 1) ? -1.0 : 1.0;
  return 2.0 * sgn * fact * (acc.re + tail.re);
}

}  // namespace mh3d
