// LDS-resident mixed-radix (8/4/2/3) Stockham FFT for gfx950 workgroups.
//
// A workgroup of T threads transforms `nlines` independent lines of length n held
// in LDS.  Element p of line l lives at buf[base(l) + p*es] with
//   base(l) = (l / l2) * s1 + (l % l2) * s2,
// which covers both "lines contiguous" and "lines interleaved" layouts and 2-D
// batches of lines.  Each radix-R stage is an out-of-place Stockham autosort step
// between two LDS buffers of the same layout (ping-pong), so a butterfly is loaded,
// twiddled, transformed and stored without holding other butterflies in registers.
// Twiddles come from an LDS table tw[t] = exp(-2 pi i t / n).
//
// Butterflies are dealt round-robin to threads; consecutive butterflies go to
// consecutive lines (lines_fast) or to consecutive positions of one line, whichever
// keeps a wavefront on consecutive LDS words.
#pragma once
#include <hip/hip_runtime.h>

namespace mh3d {

// ------------------------------------------------------------------ complex helpers
template <typename C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <typename C> __device__ __forceinline__ C cmk(typename real_of<C>::type x, typename real_of<C>::type y) {
  C c; c.x = x; c.y = y; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename C> __device__ __forceinline__ C cmulcj(C a, C b) {
  return cmk<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, typename real_of<C>::type s) {
  return cmk<C>(a.x * s, a.y * s);
}
// multiply by i*sgn (sgn = +1 or -1)
template <int SGN, typename C> __device__ __forceinline__ C cmul_i(C a) {
  return SGN > 0 ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}

// ------------------------------------------------------------------ small DFTs
// X_p = sum_q v_q exp(SGN * 2 pi i p q / R), SGN = -1 forward, +1 inverse.
template <int SGN, typename C> __device__ __forceinline__ void dft2(C* v) {
  C a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}
template <int SGN, typename C> __device__ __forceinline__ void dft3(C* v) {
  using R = typename real_of<C>::type;
  const R h = (R)0.86602540378443864676;  // sqrt(3)/2
  C s = cadd(v[1], v[2]);
  C t1 = csub(v[0], cscale(s, (R)0.5));
  C t2 = cscale(csub(v[1], v[2]), (R)SGN * h);
  v[0] = cadd(v[0], s);
  C it2 = cmk<C>(-t2.y, t2.x);  // i * t2
  v[1] = cadd(t1, it2);
  v[2] = csub(t1, it2);
}
template <int SGN, typename C> __device__ __forceinline__ void dft4(C* v) {
  C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  C a2 = cadd(v[1], v[3]), a3 = cmul_i<SGN>(csub(v[1], v[3]));
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}
template <int SGN, typename C> __device__ __forceinline__ void dft8(C* v) {
  using R = typename real_of<C>::type;
  const R r2 = (R)0.70710678118654752440;
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<SGN>(e);
  dft4<SGN>(o);
  // w^p = exp(SGN * 2 pi i p / 8)
  C w1o = cmul(o[1], cmk<C>(r2, (R)SGN * r2));
  C w2o = cmul_i<SGN>(o[2]);
  C w3o = cmul(o[3], cmk<C>(-r2, (R)SGN * r2));
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], w1o);
  v[5] = csub(e[1], w1o);
  v[2] = cadd(e[2], w2o);
  v[6] = csub(e[2], w2o);
  v[3] = cadd(e[3], w3o);
  v[7] = csub(e[3], w3o);
}
// radix 16 as two length-8 DFTs of the even and odd points and one radix-2 combination
template <int SGN, typename C> __device__ __forceinline__ void dft16(C* v) {
  using R = typename real_of<C>::type;
  const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173;   // cos, sin of pi/8
  const R r2 = (R)0.70710678118654752440;
  C e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
  dft8<SGN>(e);
  dft8<SGN>(o);
  // w^p = exp(SGN * 2 pi i p / 16), p = 0..7
  const C w[8] = {cmk<C>((R)1, (R)0), cmk<C>(c1, (R)SGN * s1), cmk<C>(r2, (R)SGN * r2), cmk<C>(s1, (R)SGN * c1),
                  cmk<C>((R)0, (R)SGN), cmk<C>(-s1, (R)SGN * c1), cmk<C>(-r2, (R)SGN * r2), cmk<C>(-c1, (R)SGN * s1)};
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const C t = p == 0 ? o[0] : cmul(o[p], w[p]);
    v[p] = cadd(e[p], t);
    v[p + 8] = csub(e[p], t);
  }
}
template <int R, int SGN, typename C> __device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 2) dft2<SGN>(v);
  else if constexpr (R == 3) dft3<SGN>(v);
  else if constexpr (R == 4) dft4<SGN>(v);
  else if constexpr (R == 16) dft16<SGN>(v);
  else dft8<SGN>(v);
}

// ------------------------------------------------------------------ radix plan and stages
struct LineMap {
  int l2, s1, s2, es;
  __device__ __forceinline__ int base(int l) const { return (l / l2) * s1 + (l % l2) * s2; }
};

// One out-of-place radix-R Stockham stage from `in` to `out` (same layout).
// ns = product of the radices already applied.  No barrier inside.
template <int R, int SGN, typename C>
__device__ __forceinline__ void fft_stage(const C* __restrict__ in, C* __restrict__ out, const C* tw, int n,
                                          int nlines, int ns, const LineMap& lm, bool lines_fast) {
  const int T = blockDim.x;
  const int nb = n / R;
  const int total = nlines * nb;
  const int twstep = n / (ns * R);
  for (int b = threadIdx.x; b < total; b += T) {
    int l, j;
    if (lines_fast) { l = b % nlines; j = b / nlines; }
    else { j = b % nb; l = b / nb; }
    const int base = lm.base(l);
    const int k = j % ns;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[base + (j + r * nb) * lm.es];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const C w = tw[k * r * twstep];
      v[r] = SGN < 0 ? cmul(v[r], w) : cmulcj(w, v[r]);
    }
    dft<R, SGN>(v);
    const int o = base + ((j / ns) * ns * R + k) * lm.es;
#pragma unroll
    for (int r = 0; r < R; ++r) out[o + r * ns * lm.es] = v[r];
  }
}

// Radix sequence of n packed 4 bits per stage (stage s in bits 4s..4s+3), 0-terminated.
__host__ __device__ inline unsigned long long radix_code(int n) {
  unsigned long long code = 0;
  int s = 0;
  while (n % 8 == 0) { code |= 8ull << (4 * s++); n /= 8; }
  while (n % 4 == 0) { code |= 4ull << (4 * s++); n /= 4; }
  while (n % 2 == 0) { code |= 2ull << (4 * s++); n /= 2; }
  while (n % 3 == 0) { code |= 3ull << (4 * s++); n /= 3; }
  return code;
}

__host__ inline bool fft_length_ok(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// Length-n transform (unnormalised) of nlines lines.  Input in *a; the stages
// ping-pong between a and b.  Returns the buffer holding the result (a or b); the
// other one is free.  All threads of the block must call it; it starts and ends
// with a barrier.
template <int SGN, typename C>
__device__ C* fft_lds(C* a, C* b, const C* tw, int n, int nlines, const LineMap& lm, bool lines_fast) {
  unsigned long long code = radix_code(n);
  int ns = 1;
  __syncthreads();
  while (code) {
    const int r = (int)(code & 15ull);
    code >>= 4;
    switch (r) {
      case 8: fft_stage<8, SGN>(a, b, tw, n, nlines, ns, lm, lines_fast); break;
      case 4: fft_stage<4, SGN>(a, b, tw, n, nlines, ns, lm, lines_fast); break;
      case 2: fft_stage<2, SGN>(a, b, tw, n, nlines, ns, lm, lines_fast); break;
      default: fft_stage<3, SGN>(a, b, tw, n, nlines, ns, lm, lines_fast); break;
    }
    __syncthreads();
    C* t = a; a = b; b = t;
    ns *= r;
  }
  return a;
}

// ------------------------------------------------------------------ compile-time lengths
// Radix of stage s for length N (same order as radix_code: 8s, 4s, 2s, 3s).
__host__ __device__ constexpr int ct_radix(int n, int s) {
  int i = 0;
  while (n % 8 == 0) { if (i == s) return 8; n /= 8; ++i; }
  while (n % 4 == 0) { if (i == s) return 4; n /= 4; ++i; }
  while (n % 2 == 0) { if (i == s) return 2; n /= 2; ++i; }
  while (n % 3 == 0) { if (i == s) return 3; n /= 3; ++i; }
  return 0;
}

// One out-of-place stage for compile-time N, radix R and NS (product of previous
// radices).  Lines are contiguous: element p of line l at l*ls + p.  Consecutive
// butterflies of a line go to consecutive lanes.
template <int N, int R, int NS, int SGN, typename C>
__device__ __forceinline__ void ct_stage(const C* __restrict__ in, C* __restrict__ out, const C* tw,
                                         int nlines, int ls) {
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
  const int total = nlines * NB;
  for (int b = threadIdx.x; b < total; b += blockDim.x) {
    const int l = b / NB, j = b - (b / NB) * NB;
    const int k = j % NS;
    const int base = l * ls;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = in[base + j + r * NB];
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tw[k * r * TWS];
        v[r] = SGN < 0 ? cmul(v[r], w) : cmulcj(w, v[r]);
      }
    }
    dft<R, SGN>(v);
    const int o = base + (j / NS) * NS * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) out[o + r * NS] = v[r];
  }
}

template <int N, int S, int NS, int SGN, typename C>
__device__ __forceinline__ C* ct_stages(C* a, C* b, const C* tw, int nlines, int ls) {
  constexpr int R = ct_radix(N, S);
  if constexpr (R == 0) {
    return a;
  } else {
    ct_stage<N, R, NS, SGN>(a, b, tw, nlines, ls);
    __syncthreads();
    return ct_stages<N, S + 1, NS * R, SGN>(b, a, tw, nlines, ls);
  }
}

// Length-n transform of nlines contiguous lines (line stride ls) with the length
// dispatched to a compile-time instantiation when it is one of the common sizes,
// else to the runtime engine.  Same contract as fft_lds.
template <int SGN, typename C>
__device__ C* fft_lines(C* a, C* b, const C* tw, int n, int nlines, int ls) {
  __syncthreads();
  switch (n) {
#define MH3D_CT(NN) case NN: return ct_stages<NN, 0, 1, SGN>(a, b, tw, nlines, ls);
    MH3D_CT(2) MH3D_CT(3) MH3D_CT(4) MH3D_CT(6) MH3D_CT(8) MH3D_CT(12) MH3D_CT(16) MH3D_CT(24)
    MH3D_CT(32) MH3D_CT(48) MH3D_CT(64) MH3D_CT(96) MH3D_CT(128) MH3D_CT(192) MH3D_CT(256)
#undef MH3D_CT
    default: return fft_lds<SGN>(a, b, tw, n, nlines, LineMap{nlines, 0, ls, 1}, false);
  }
}

// Global-memory loads and stores through address-space-1 pointers.  A pointer read from
// a descriptor in memory is generic to the compiler, which then emits flat instructions;
// those count against the LDS counter as well, so every later LDS wait (each transform
// stage has one) would also wait for them.  HIP's vector types are classes whose copies
// go through a generic this pointer, so the accesses use clang's native vectors.
typedef float gvec2 __attribute__((ext_vector_type(2)));
typedef float gvec4 __attribute__((ext_vector_type(4)));
#define MH3D_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ldg(const T* p) { return *p; }
__device__ __forceinline__ float ldg(const float* p) { return *(const MH3D_GLOBAL float*)p; }
__device__ __forceinline__ float2 ldg(const float2* p) {
  const gvec2 v = *(const MH3D_GLOBAL gvec2*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float4 ldg(const float4* p) {
  const gvec4 v = *(const MH3D_GLOBAL gvec4*)p;
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stg(float* p, float v) { *(MH3D_GLOBAL float*)p = v; }
__device__ __forceinline__ void stg(float2* p, float2 v) {
  gvec2 w;
  w.x = v.x;
  w.y = v.y;
  *(MH3D_GLOBAL gvec2*)p = w;
}
__device__ __forceinline__ void stg(float4* p, float4 v) {
  gvec4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *(MH3D_GLOBAL gvec4*)p = w;
}

// Copy a length-n twiddle table from global memory into LDS (then barrier by caller).
template <typename C>
__device__ __forceinline__ void load_table(C* dst, const C* src, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) dst[t] = ldg(src + t);
}

}  // namespace mh3d
