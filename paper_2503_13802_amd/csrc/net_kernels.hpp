// Warm-start 3D U-Net on gfx950: BF16 activations and weights, FP32 accumulation on
// MFMA (v_mfma_f32_16x16x32_bf16, two 16-deep reduction chunks per instruction; a
// trailing odd chunk uses v_mfma_f32_16x16x16_bf16), FP32 master weights, Adam.
//
// Tensors are channels-last BF16 [X][Y][Z][Cs] with the channel stride Cs a
// multiple of 4 (padding channels hold zeros).  Grid axes are powers of two so
// voxel decoding is shifts.  A 3x3x3 convolution is an implicit GEMM
//   out[n][co] = b[co] + sum_k W[co][k] in[n + d(tap(k))][ci(k)],  k = tap*Cs_in + ci,
// tap = (dx+1)*9 + (dy+1)*3 + (dz+1), zero outside the grid; K is padded to a
// multiple of 16 with zero weights.  One wavefront computes 16 voxels x all output
// channels (16-wide tiles); per MFMA the lane layout is
//   A[row = lane%16][k = 4*(lane/16) + j]   (voxel x reduction),
//   B[k = 4*(lane/16) + j][col = lane%16]   (reduction x channel),
//   D[row = 4*(lane/16) + j][col = lane%16].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mh3d {
namespace net {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Two 16-deep reduction chunks in one 16x16x32 MFMA.  The instruction reads lane group g
// (lane / 16) element j as reduction index 8g + j of A and of B; placing chunk 0's
// slice (k = 4g + j) in elements 0..3 and chunk 1's (k = 16 + 4g + j) in 4..7 applies
// the same permutation of the 32 reduction indices to both operands, so the result is
// the sum of the two 16x16x16 products (in another order of the FP32 additions).
__device__ __forceinline__ f4v mfma2(s4v a0, s4v a1, s4v b0, s4v b1, f4v c) {
  const s8v a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
  const s8v b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
}

constexpr int NT_MAX = 7;   // output-channel tiles per wave (112 channels)

// FP32 -> BF16, round to nearest even (NaN kept quiet).
// Nearest BF16, ties to even (gfx950's v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct Dims {
  int lx, ly, lz;          // log2 of the axes
  __host__ __device__ __forceinline__ long long n() const { return 1ll << (lx + ly + lz); }
  __device__ __forceinline__ void decode(long long i, int& x, int& y, int& z) const {
    z = (int)(i & ((1ll << lz) - 1));
    y = (int)((i >> lz) & ((1ll << ly) - 1));
    x = (int)(i >> (ly + lz));
  }
  __device__ __forceinline__ long long encode(int x, int y, int z) const {
    return ((long long)x << (ly + lz)) | ((long long)y << lz) | z;
  }
  __device__ __forceinline__ bool inside(int x, int y, int z) const {
    return x >= 0 && y >= 0 && z >= 0 && x < (1 << lx) && y < (1 << ly) && z < (1 << lz);
  }
};

__device__ __forceinline__ void tap_offset(int tap, int ks, int& dx, int& dy, int& dz) {
  if (ks == 1) { dx = dy = dz = 0; return; }
  dx = tap / 9 - 1;
  dy = (tap / 3) % 3 - 1;
  dz = tap % 3 - 1;
}

// Convolution (ks = 3 or 1).  in: [N][cs_in]; W: [cout_tiles*16][kp] BF16; bias FP32
// [cout]; out: BF16 [N][cs_out] or FP32 [N] (OUTF32, cout == 1).  Padding output
// channels cout..cs_out-1 are written as zeros.  block = 256 (4 waves, 64 voxels).
template <bool RELU, bool OUTF32>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ in, Dims dm, int cs_in, int ks,
                                              const uint16_t* __restrict__ W, int kp,
                                              const float* __restrict__ bias, int cout, int cs_out,
                                              void* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long N = dm.n();
  const long long n0 = ((long long)blockIdx.x * 4 + wave) * 16;
  if (n0 >= N) return;                      // wave-uniform, no block barriers below
  const int r = lane & 15, g = lane >> 4;
  const long long n = n0 + r;
  const bool nvalid = n < N;
  int x = 0, y = 0, z = 0;
  if (nvalid) dm.decode(n, x, y, z);
  const int ntile = (cout + 15) >> 4;
  const int ntap = ks * ks * ks;
  f4v acc[NT_MAX];
#pragma unroll
  for (int t = 0; t < NT_MAX; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  int tap = 0, ci = 4 * g;
  while (ci >= cs_in) { ci -= cs_in; ++tap; }
  // A slice of the current chunk (this lane's voxel, 4 reduction indices), then step
  auto a_next = [&]() {
    s4v a = s4v{0, 0, 0, 0};
    if (nvalid && tap < ntap) {
      int dx, dy, dz;
      tap_offset(tap, ks, dx, dy, dz);
      const int xx = x + dx, yy = y + dy, zz = z + dz;
      if (dm.inside(xx, yy, zz)) a = *reinterpret_cast<const s4v*>(in + dm.encode(xx, yy, zz) * cs_in + ci);
    }
    ci += 16;
    while (ci >= cs_in) { ci -= cs_in; ++tap; }
    return a;
  };
  const int nkc = kp >> 4;
  for (int kc = 0; kc < nkc; kc += 2) {
    const s4v a0 = a_next();
    const uint16_t* wr = W + (long long)r * kp + kc * 16 + 4 * g;
    if (kc + 1 < nkc) {
      const s4v a1 = a_next();
#pragma unroll
      for (int t = 0; t < NT_MAX; ++t) {
        if (t < ntile) {
          const s4v b0 = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp);
          const s4v b1 = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp + 16);
          acc[t] = mfma2(a0, a1, b0, b1, acc[t]);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT_MAX; ++t) {
        if (t < ntile) {
          const s4v b = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b, acc[t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT_MAX; ++t) {
    if (t >= ntile) break;
    const int co = t * 16 + r;
    const float bv = co < cout ? bias[co] : 0.f;   // once: the stores may alias bias for the compiler
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long nn = n0 + 4 * g + j;
      if (nn >= N) continue;
      if constexpr (OUTF32) {
        if (co == 0) reinterpret_cast<float*>(out)[nn] = acc[t][j] + bv;
      } else {
        if (co < cout) {
          float v = acc[t][j] + bv;
          if (RELU) v = fmaxf(v, 0.f);
          reinterpret_cast<uint16_t*>(out)[nn * cs_out + co] = f2bf(v);
        } else if (co < cs_out) {
          reinterpret_cast<uint16_t*>(out)[nn * cs_out + co] = 0;
        }
      }
    }
  }
}

// Convolution with the reduction split over the 4 waves of a block (for deep K on
// small grids, where k_conv has too few waves to hide its load latency): the block
// owns 16 voxels, wave w takes the K chunks w, w+4, ..., the partial tiles are
// summed in LDS in wave order and wave 0 writes the result.  Same operands, output
// and padding rules as k_conv (BF16 output).  grid = ceil(N/16), block = 256.
template <bool RELU>
__global__ __launch_bounds__(256) void k_conv_splitk(const uint16_t* __restrict__ in, Dims dm, int cs_in, int ks,
                                                     const uint16_t* __restrict__ W, int kp,
                                                     const float* __restrict__ bias, int cout, int cs_out,
                                                     uint16_t* __restrict__ out) {
  __shared__ f4v part[3][NT_MAX][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long N = dm.n();
  const long long n0 = (long long)blockIdx.x * 16;
  const int r = lane & 15, g = lane >> 4;
  const long long n = n0 + r;
  const bool nvalid = n < N;
  int x = 0, y = 0, z = 0;
  if (nvalid) dm.decode(n, x, y, z);
  const int ntile = (cout + 15) >> 4;
  const int ntap = ks * ks * ks;
  f4v acc[NT_MAX];
#pragma unroll
  for (int t = 0; t < NT_MAX; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  // k = kc*16 + 4g: start at chunk `wave`, step 4 chunks (64 k) at a time
  int tap = 0, ci = wave * 16 + 4 * g;
  while (ci >= cs_in) { ci -= cs_in; ++tap; }
  // A slice of this wave's current chunk, then step to its next chunk (4 chunks on)
  auto a_next = [&]() {
    s4v a = s4v{0, 0, 0, 0};
    if (nvalid && tap < ntap) {
      int dx, dy, dz;
      tap_offset(tap, ks, dx, dy, dz);
      const int xx = x + dx, yy = y + dy, zz = z + dz;
      if (dm.inside(xx, yy, zz)) a = *reinterpret_cast<const s4v*>(in + dm.encode(xx, yy, zz) * cs_in + ci);
    }
    ci += 64;
    while (ci >= cs_in) { ci -= cs_in; ++tap; }
    return a;
  };
  const int nkc = kp >> 4;
  for (int kc = wave; kc < nkc; kc += 8) {   // chunks kc and kc + 4 in one instruction
    const s4v a0 = a_next();
    const uint16_t* wr = W + (long long)r * kp + kc * 16 + 4 * g;
    if (kc + 4 < nkc) {
      const s4v a1 = a_next();
#pragma unroll
      for (int t = 0; t < NT_MAX; ++t) {
        if (t < ntile) {
          const s4v b0 = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp);
          const s4v b1 = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp + 64);
          acc[t] = mfma2(a0, a1, b0, b1, acc[t]);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT_MAX; ++t) {
        if (t < ntile) {
          const s4v b = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b, acc[t], 0, 0, 0);
        }
      }
    }
  }
  if (wave) {
#pragma unroll
    for (int t = 0; t < NT_MAX; ++t)
      if (t < ntile) part[wave - 1][t][lane] = acc[t];
  }
  __syncthreads();
  if (wave) return;
#pragma unroll
  for (int t = 0; t < NT_MAX; ++t) {
    if (t >= ntile) break;
    f4v v = acc[t];
#pragma unroll
    for (int w = 0; w < 3; ++w) v += part[w][t][lane];
    const int co = t * 16 + r;
    const float bv = co < cout ? bias[co] : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long nn = n0 + 4 * g + j;
      if (nn >= N) continue;
      if (co < cout) {
        float o = v[j] + bv;
        if (RELU) o = fmaxf(o, 0.f);
        out[nn * cs_out + co] = f2bf(o);
      } else if (co < cs_out) {
        out[nn * cs_out + co] = 0;
      }
    }
  }
}

// The 6 x 6 x 18 input halo of a 4 x 4 x 16 output tile at (x0, y0, z0) into LDS
// ([voxel][cs_in], zero outside the volume), 4 channels (8 bytes) per item with z-runs
// contiguous in global memory.  A thread's items go in batches of 8 whose loads are all
// issued before the LDS writes (a load-then-write loop would wait on every load).
__device__ __forceinline__ void stage_halo(uint16_t* __restrict__ tile, const uint16_t* __restrict__ in, const Dims& dm,
                                           int cs_in, int x0, int y0, int z0) {
  const int cq = cs_in >> 2;
  const int nitem = 648 * cq;
  for (int q0 = threadIdx.x; q0 < nitem; q0 += 8 * 256) {
    s4v val[8];
    int dst[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + u * 256;
      val[u] = s4v{0, 0, 0, 0};
      dst[u] = -1;
      if (q < nitem) {
        const int v = q / cq, c4 = q - v * cq;
        const int zl = v % 18, yl = (v / 18) % 6, xl = v / 108;
        const int gx = x0 + xl - 1, gy = y0 + yl - 1, gz = z0 + zl - 1;
        dst[u] = v * cs_in + 4 * c4;
        if (dm.inside(gx, gy, gz)) val[u] = *reinterpret_cast<const s4v*>(in + dm.encode(gx, gy, gz) * cs_in + 4 * c4);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (dst[u] >= 0) *reinterpret_cast<s4v*>(tile + dst[u]) = val[u];
  }
}

// k_conv_splitk for input channel strides divisible by 8: MFMA m takes the reduction
// indices 32 m .. 32 m + 31, lane group g the 8 consecutive channels 32 m + 8 g .. + 7 of
// one tap (one 16-byte gather of A, one 16-byte load of B per output tile); wave w takes
// m = w, w + 4, ..., U of them with all their loads issued before their MFMAs.
template <bool RELU, int NT>
__global__ __launch_bounds__(256) void k_conv_splitk8(const uint16_t* __restrict__ in, Dims dm, int cs_in, int ks,
                                                      const uint16_t* __restrict__ W, int kp,
                                                      const float* __restrict__ bias, int cout, int cs_out,
                                                      uint16_t* __restrict__ out) {
  constexpr int U = NT <= 2 ? 4 : 2;   // loads in flight per wave: U gathers and U * NT weight slices
  __shared__ f4v part[3][NT][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long N = dm.n();
  const long long n0 = (long long)blockIdx.x * 16;
  const int r = lane & 15, g = lane >> 4;
  const long long n = n0 + r;
  const bool nvalid = n < N;
  int x = 0, y = 0, z = 0;
  if (nvalid) dm.decode(n, x, y, z);
  const int ntap = ks * ks * ks;
  f4v acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f4v{0.f, 0.f, 0.f, 0.f};
  // k = 32 m + 8 g for m = wave + 4 i: start, then step 128 reduction indices
  int tap = 0, ci = 32 * wave + 8 * g;
  while (ci >= cs_in) { ci -= cs_in; ++tap; }
  const int nm = (kp + 31) >> 5;
  const uint16_t* wr = W + (long long)r * kp + 8 * g;
  for (int m0 = wave; m0 < nm; m0 += 4 * U) {
    s8v a[U], b[U][NT];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int m = m0 + 4 * u;
      a[u] = s8v{0, 0, 0, 0, 0, 0, 0, 0};
      if (m < nm && nvalid && tap < ntap) {
        int dx, dy, dz;
        tap_offset(tap, ks, dx, dy, dz);
        const int xx = x + dx, yy = y + dy, zz = z + dz;
        if (dm.inside(xx, yy, zz)) a[u] = *reinterpret_cast<const s8v*>(in + dm.encode(xx, yy, zz) * cs_in + ci);
      }
      const bool kin = m < nm && 32 * m + 8 * g < kp;
#pragma unroll
      for (int t = 0; t < NT; ++t)
        b[u][t] = kin ? *reinterpret_cast<const s8v*>(wr + (long long)t * 16 * kp + 32 * m) : s8v{0, 0, 0, 0, 0, 0, 0, 0};
      ci += 128;
      while (ci >= cs_in) { ci -= cs_in; ++tap; }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a[u]), __builtin_bit_cast(bf8v, b[u][t]),
                                                           acc[t], 0, 0, 0);
  }
  if (wave) {
#pragma unroll
    for (int t = 0; t < NT; ++t) part[wave - 1][t][lane] = acc[t];
  }
  __syncthreads();
  if (wave) return;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    f4v v = acc[t];
#pragma unroll
    for (int w = 0; w < 3; ++w) v += part[w][t][lane];
    const int co = t * 16 + r;
    const float bv = co < cout ? bias[co] : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long nn = n0 + 4 * g + j;
      if (nn >= N) continue;
      if (co < cout) {
        float o = v[j] + bv;
        if (RELU) o = fmaxf(o, 0.f);
        out[nn * cs_out + co] = f2bf(o);
      } else if (co < cs_out) {
        out[nn * cs_out + co] = 0;
      }
    }
  }
}

// 3x3x3 convolution on an LDS-staged tile with the input channel stride CS fixed at
// compile time (the same implicit GEMM, tile and operands as k_conv_tiled, kp = 16
// NKC).  Every index the reduction needs is a constant or comes from a per-block table
// of the 4 lane groups' offsets per K chunk, so the reduction costs an LDS read of the
// offset, the operand reads at immediate offsets and the MFMA: no tap arithmetic per
// chunk.  The halo goes in per voxel (one contiguous CS-channel run), and the output
// tile leaves through LDS as contiguous 16- or 8-byte pieces of each z-run.
// C1 > 0: the input is the decoder's concatenation [skip, upsampled coarse] read in place
// (no concatenated copy): channels [0, C1) of voxel n from `in` (stride C1), the other
// CS - C1 from `in2` (stride CS - C1) at the coarse voxel (x/2, y/2, z/2), the halo
// tile holding the same values the concatenated tensor would.
template <int CS, int NT, bool RELU, int C1 = 0>
__global__ __launch_bounds__(256) void k_conv_ct(const uint16_t* __restrict__ in, Dims dm,
                                                 const uint16_t* __restrict__ W, int kp,
                                                 const float* __restrict__ bias, int cout, int cs_out,
                                                 uint16_t* __restrict__ out, const uint16_t* __restrict__ in2) {
  static_assert(C1 % 4 == 0 && C1 < CS, "the skip channels are whole 4-channel groups");
  constexpr int NKC = (27 * CS + 15) / 16;
  constexpr int RS = 18 * CS;                       // one (x, y) row of the halo
  constexpr int HALO = 648 * CS;
  constexpr int STAGE = 256 * 16 * NT;              // output staging (elements), at most
  constexpr int TILE = ((HALO > STAGE ? HALO : STAGE) + 7) & ~7;
  extern __shared__ uint16_t sm[];
  uint16_t* tile = sm;
  int* toff = reinterpret_cast<int*>(sm + TILE);   // [NKC][4] element offsets
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int nzt = dm.lz - 4, nyt = dm.ly - 2;
  const int tz = blockIdx.x & ((1 << nzt) - 1);
  const int rest = blockIdx.x >> nzt;
  const int ty = rest & ((1 << nyt) - 1);
  const int tx = rest >> nyt;
  const int x0 = tx * 4, y0 = ty * 4, z0 = tz * 16;
  // reduction index k = 16 kc + 4 g + j -> (tap, channel) -> halo offset; the padding
  // columns (tap >= 27) meet zero rows of W and read any finite halo entry (offset 0)
  // (CS % 8 == 0: entry m * 4 + g holds k = 32 m + 8 g; else entry kc * 4 + g, k = 16 kc + 4 g)
  constexpr int NTAB = CS % 8 == 0 ? 4 * ((16 * NKC + 31) / 32) : 4 * NKC;
  for (int i = threadIdx.x; i < NTAB; i += 256) {
    const int k = (CS % 8 == 0 ? 8 : 4) * i;
    const int tap = k / CS, ci = k - (k / CS) * CS;
    toff[i] = tap < 27 ? ((tap / 9) * 108 + ((tap / 3) % 3) * 18 + tap % 3) * CS + ci : 0;
  }
  // halo: voxel v = threadIdx.x + 256 u, its CS channels as CS/4 8-byte loads, all of a
  // thread's loads issued before its LDS writes
  {
    constexpr int NQ = CS / 4, NQ1 = C1 / 4;
    const Dims dc{dm.lx - 1, dm.ly - 1, dm.lz - 1};
    s4v val[3][NQ];
    long long src[3], src2[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int v = threadIdx.x + 256 * u;
      src[u] = -1;
      src2[u] = 0;
      if (v < 648) {
        const int zl = v % 18, yl = (v / 18) % 6, xl = v / 108;
        const int gx = x0 + xl - 1, gy = y0 + yl - 1, gz = z0 + zl - 1;
        if (dm.inside(gx, gy, gz)) {
          src[u] = dm.encode(gx, gy, gz) * (C1 > 0 ? C1 : CS);
          if constexpr (C1 > 0) src2[u] = dc.encode(gx >> 1, gy >> 1, gz >> 1) * (CS - C1);
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const uint16_t* p = (C1 > 0 && q >= NQ1) ? in2 + src2[u] + 4 * (q - NQ1) : in + src[u] + 4 * q;
        val[u][q] = src[u] >= 0 ? *reinterpret_cast<const s4v*>(p) : s4v{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int v = threadIdx.x + 256 * u;
      if (v < 648) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) *reinterpret_cast<s4v*>(tile + v * CS + 4 * q) = val[u][q];
      }
    }
  }
  __syncthreads();
  const int lbase = (wave * 108 + r) * CS;
  f4v acc[4][NT];
#pragma unroll
  for (int yy = 0; yy < 4; ++yy)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[yy][t] = f4v{0.f, 0.f, 0.f, 0.f};
  if constexpr (CS % 8 == 0) {
    // lane group g takes the 8 consecutive reduction indices 32 m + 8 g .. + 7 of MFMA m:
    // 8 channels of one tap, one 16-byte LDS read of A and one 16-byte load of B (the
    // same index on both operands); W's padding columns (k >= 16 NKC) read as zeros
    constexpr int KP = 16 * NKC, NM = (KP + 31) / 32;
    const uint16_t* wr8 = W + (long long)r * KP + 8 * g;
#pragma unroll 4
    for (int m = 0; m < NM; ++m) {
      const int o = lbase + toff[m * 4 + g];
      s8v b[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        b[t] = (32 * m + 8 * g < KP) ? *reinterpret_cast<const s8v*>(wr8 + t * 16 * KP + 32 * m)
                                     : s8v{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int yy = 0; yy < 4; ++yy) {
        const s8v av = *reinterpret_cast<const s8v*>(tile + o + yy * RS);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[yy][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, av),
                                                               __builtin_bit_cast(bf8v, b[t]), acc[yy][t], 0, 0, 0);
      }
    }
  } else {
  const uint16_t* wr = W + (long long)r * kp + 4 * g;
  auto pair = [&](int kc, bool two) {
    const int o0 = lbase + toff[kc * 4 + g];
    const int o1 = two ? lbase + toff[(kc + 1) * 4 + g] : 0;
    s4v b0[NT], b1[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      b0[t] = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp + kc * 16);
      b1[t] = two ? *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp + kc * 16 + 16) : s4v{0, 0, 0, 0};
    }
#pragma unroll
    for (int yy = 0; yy < 4; ++yy) {
      const s4v a0 = *reinterpret_cast<const s4v*>(tile + o0 + yy * RS);
      const s4v a1 = two ? *reinterpret_cast<const s4v*>(tile + o1 + yy * RS) : s4v{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[yy][t] = mfma2(a0, a1, b0[t], b1[t], acc[yy][t]);
    }
  };
#pragma unroll 4
  for (int kc = 0; kc + 1 < NKC; kc += 2) pair(kc, true);
  if constexpr (NKC & 1) pair(NKC - 1, false);
  }
  __syncthreads();   // every wave is done with the halo: its space stages the output
  // D[row = 4g + j][col = r]: voxel z0 + 4g + j of row (x0 + wave, y0 + yy), channel t*16 + r
  uint16_t* st = tile + wave * 64 * cs_out;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int co = t * 16 + r;
    const bool live = co < cout;
    const float bv = live ? bias[co] : 0.f;
    if (co < cs_out) {
      uint16_t* sl = st + 4 * g * cs_out + co;
#pragma unroll
      for (int yy = 0; yy < 4; ++yy)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float v = acc[yy][t][j] + bv;
          if (RELU) v = fmaxf(v, 0.f);
          const uint16_t h = f2bf(v);
          sl[(yy * 16 + j) * cs_out] = live ? h : (uint16_t)0;
        }
    }
  }
  __syncthreads();
  // each (x, y) row of 16 voxels is a contiguous run of 16 cs_out channels in memory: the
  // wave's 4 rows as 16-byte (8-byte) pieces, piece p of row p / per_row
  const long long row0 = dm.encode(x0 + wave, y0, z0) * cs_out;
  const long long ystride = (long long)cs_out << (dm.lz);   // one y step, in elements
  if ((cs_out & 7) == 0) {
    const int per_row = 2 * cs_out;
    for (int p = lane; p < 4 * per_row; p += 64) {
      const int yy = p / per_row, q = p - yy * per_row;
      *reinterpret_cast<uint4*>(out + row0 + yy * ystride + 8 * q) =
          *reinterpret_cast<const uint4*>(st + yy * 16 * cs_out + 8 * q);
    }
  } else {
    const int per_row = 4 * cs_out;
    for (int p = lane; p < 4 * per_row; p += 64) {
      const int yy = p / per_row, q = p - yy * per_row;
      *reinterpret_cast<s4v*>(out + row0 + yy * ystride + 4 * q) =
          *reinterpret_cast<const s4v*>(st + yy * 16 * cs_out + 4 * q);
    }
  }
}

// LDS bytes of k_conv_ct<CS, NT, *>.
template <int CS, int NT>
constexpr size_t conv_ct_lds() {
  constexpr int NKC = (27 * CS + 15) / 16;
  constexpr int HALO = 648 * CS, STAGE = 256 * 16 * NT;
  constexpr int TILE = ((HALO > STAGE ? HALO : STAGE) + 7) & ~7;
  return sizeof(uint16_t) * TILE + sizeof(int) * NKC * 4;   // the table of either layout fits in NKC * 4
}

// 3x3x3 convolution on an LDS-staged input tile (the same implicit GEMM as k_conv).
// A workgroup of 4 waves computes a 4 (x) x 4 (y) x 16 (z) output tile: the input
// block with its one-voxel halo, 6 x 6 x 18 voxels x cs_in channels (zero outside
// the grid), is loaded once into LDS and every tap reads the A operand from there;
// wave w takes x = x0 + w and four 16-voxel z rows (y = y0 .. y0+3), so each weight
// fragment feeds 4 x NT MFMAs.  Needs lz >= 4, ly >= 2, lx >= 2 and NT*16 >= cout.
// grid = (X/4)(Y/4)(Z/16), block = 256, dynamic LDS = 648 cs_in BF16.
template <bool RELU, int NT>
__global__ __launch_bounds__(256) void k_conv_tiled(const uint16_t* __restrict__ in, Dims dm, int cs_in,
                                                    const uint16_t* __restrict__ W, int kp,
                                                    const float* __restrict__ bias, int cout, int cs_out,
                                                    uint16_t* __restrict__ out) {
  extern __shared__ uint16_t tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nzt = dm.lz - 4, nyt = dm.ly - 2;
  const int tz = blockIdx.x & ((1 << nzt) - 1);
  const int rest = blockIdx.x >> nzt;
  const int ty = rest & ((1 << nyt) - 1);
  const int tx = rest >> nyt;
  const int x0 = tx * 4, y0 = ty * 4, z0 = tz * 16;
  stage_halo(tile, in, dm, cs_in, x0, y0, z0);
  __syncthreads();
  const int r = lane & 15, g = lane >> 4;
  f4v acc[4][NT];
#pragma unroll
  for (int yy = 0; yy < 4; ++yy)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[yy][t] = f4v{0.f, 0.f, 0.f, 0.f};
  int tap = 0, ci = 4 * g;
  while (ci >= cs_in) { ci -= cs_in; ++tap; }
  const int row_stride = 18 * cs_in;            // one (x, y) row of the tile
  // LDS offset of the current chunk's A slice (taps past 26 only meet the zero padding
  // rows of W: their A values stay 0, offset -1), then step to the next chunk
  auto off_next = [&]() {
    int off = -1;
    if (tap < 27) {
      const int dx = tap / 9, dy = (tap / 3) % 3, dz = tap % 3;
      off = ((wave + dx) * 6 + dy) * row_stride + (r + dz) * cs_in + ci;
    }
    ci += 16;
    while (ci >= cs_in) { ci -= cs_in; ++tap; }
    return off;
  };
  auto a_at = [&](int off, int yy) {
    return off >= 0 ? *reinterpret_cast<const s4v*>(tile + off + yy * row_stride) : s4v{0, 0, 0, 0};
  };
  const int nkc = kp >> 4;
  const uint16_t* wr = W + (long long)r * kp + 4 * g;
  // B slices of the chunk pair (kc, kc + 1), loaded one pair ahead; an odd last chunk
  // pairs with zeros (its products add exact zeros)
  s4v nb0[NT], nb1[NT];
  auto load_b = [&](int kc) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      nb0[t] = *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp + kc * 16);
      nb1[t] = kc + 1 < nkc ? *reinterpret_cast<const s4v*>(wr + (long long)t * 16 * kp + kc * 16 + 16) : s4v{0, 0, 0, 0};
    }
  };
  load_b(0);
  for (int kc = 0; kc < nkc; kc += 2) {
    s4v b0[NT], b1[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) { b0[t] = nb0[t]; b1[t] = nb1[t]; }
    if (kc + 2 < nkc) load_b(kc + 2);
    const int off0 = off_next();
    const int off1 = kc + 1 < nkc ? off_next() : -1;
#pragma unroll
    for (int yy = 0; yy < 4; ++yy) {
      const s4v a0 = a_at(off0, yy), a1 = a_at(off1, yy);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[yy][t] = mfma2(a0, a1, b0[t], b1[t], acc[yy][t]);
    }
  }
  // D[row = 4g + j][col = r]: voxel z0 + 4g + j of row (x0 + wave, y0 + yy), channel t*16 + r
#pragma unroll
  for (int yy = 0; yy < 4; ++yy) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + r;
      const float bv = co < cout ? bias[co] : 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long nn = dm.encode(x0 + wave, y0 + yy, z0 + 4 * g + j);
        if (co < cout) {
          float v = acc[yy][t][j] + bv;
          if (RELU) v = fmaxf(v, 0.f);
          out[nn * cs_out + co] = f2bf(v);
        } else if (co < cs_out) {
          out[nn * cs_out + co] = 0;
        }
      }
    }
  }
}

// Weight gradient of a 3x3x3 layer on LDS-staged tiles:
//   gW[co][k] += sum_n gout[n][co] in[n + d(tap(k))][ci(k)].
// A block walks tpb consecutive 4 x 4 x 16 voxel tiles; per tile it stages the input
// block with its halo (as k_conv_tiled) and the output gradient transposed to
// [co][voxel] (rows up to 16*ceil(cout/16), the padding rows zero).  Its 16 output
// blocks of 16 (co) x 16 (k) -- blockIdx.y selects which -- are spread 4 per wave;
// per 16-voxel row an MFMA takes A[co][v] = gout[v][co], B[v][k] = in-patch[v][k].
// The FP32 sums stay in registers over the tiles, then one atomic add per value.
// grid = (ceil(tiles / tpb), ceil(blocks / 16)), block = 256,
// dynamic LDS = (648 cs_in + 256 * 16 ceil(cout/16)) BF16.
__global__ __launch_bounds__(256) void k_conv_wgrad_tiled(const uint16_t* __restrict__ in, Dims dm, int cs_in,
                                                          const uint16_t* __restrict__ gout, int cs_g, int cout,
                                                          int kp, float* __restrict__ gW, int tpb) {
  extern __shared__ uint16_t sm[];
  const int ncot = (cout + 15) >> 4, nkc = kp >> 4, nblk = ncot * nkc;
  uint16_t* halo = sm;
  uint16_t* gT = sm + 648 * cs_in;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g4 = lane >> 4;
  const int nzt = dm.lz - 4, nyt = dm.ly - 2;
  const int ntiles = (int)(dm.n() >> 8);
  // this wave's four blocks and, per lane, the column k = kc*16 + r of each
  int bco[4], bkc[4], boff[4];
  bool bval[4], tval[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = blockIdx.y * 16 + wave * 4 + i;
    bval[i] = b < nblk;
    bco[i] = bval[i] ? b % ncot : 0;
    bkc[i] = bval[i] ? b / ncot : 0;
    const int k = bkc[i] * 16 + r;
    const int tap = k / cs_in, ci = k - tap * cs_in;
    tval[i] = bval[i] && tap < 27;
    boff[i] = tval[i] ? (((tap / 9) * 6 + (tap / 3) % 3) * 18 + tap % 3) * cs_in + ci : 0;
  }
  f4v acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f4v{0.f, 0.f, 0.f, 0.f};
  // padding rows of the transposed gradient stay zero for every tile
  for (int q = threadIdx.x; q < (ncot * 16 - cs_g) * 256; q += 256) gT[cs_g * 256 + q] = 0;
  const int cqg = cs_g >> 2;
  for (int it = 0; it < tpb; ++it) {
    const int tile = blockIdx.x * tpb + it;
    if (tile >= ntiles) break;
    const int tz = tile & ((1 << nzt) - 1), rest = tile >> nzt;
    const int ty = rest & ((1 << nyt) - 1), tx = rest >> nyt;
    const int x0 = tx * 4, y0 = ty * 4, z0 = tz * 16;
    __syncthreads();      // the previous tile's reads are done
    stage_halo(halo, in, dm, cs_in, x0, y0, z0);
    {
      // the tile's output gradients, transposed to [channel][voxel]: thread = voxel v,
      // its cqg loads issued (in batches of 8) before the LDS writes
      const int v = threadIdx.x;
      const long long nn = dm.encode(x0 + (v >> 6), y0 + ((v >> 4) & 3), z0 + (v & 15));
      for (int c0 = 0; c0 < cqg; c0 += 8) {
        s4v val[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (c0 + u < cqg) val[u] = *reinterpret_cast<const s4v*>(gout + nn * cs_g + 4 * (c0 + u));
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (c0 + u < cqg) {
#pragma unroll
            for (int j = 0; j < 4; ++j) gT[(4 * (c0 + u) + j) * 256 + v] = (uint16_t)val[u][j];
          }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int vc = 0; vc < 16; vc += 2) {   // 16-voxel rows vc and vc + 1 in one instruction
      // voxels v = vc*16 + 4*g4 + j: row (xl, yl) = (vc / 4, vc % 4), z = 4*g4 + j
      const int rowoff0 = ((vc >> 2) * 6 + (vc & 3)) * 18 * cs_in + 4 * g4 * cs_in;
      const int rowoff1 = (((vc + 1) >> 2) * 6 + ((vc + 1) & 3)) * 18 * cs_in + 4 * g4 * cs_in;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (!bval[i]) continue;
        const uint16_t* ar = gT + (bco[i] * 16 + r) * 256 + vc * 16 + 4 * g4;
        const s4v a0 = *reinterpret_cast<const s4v*>(ar);
        const s4v a1 = *reinterpret_cast<const s4v*>(ar + 16);
        s4v b0 = s4v{0, 0, 0, 0}, b1 = s4v{0, 0, 0, 0};
        if (tval[i]) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            b0[j] = (short)halo[boff[i] + rowoff0 + j * cs_in];
            b1[j] = (short)halo[boff[i] + rowoff1 + j * cs_in];
          }
        }
        acc[i] = mfma2(a0, a1, b0, b1, acc[i]);
      }
    }
  }
  // D[row = 4*g4 + j][col = r] -> (co = bco*16 + 4*g4 + j, k = bkc*16 + r)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!bval[i]) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = bco[i] * 16 + 4 * g4 + j;
      if (co < cout && acc[i][j] != 0.f) atomicAdd(&gW[(long long)co * kp + bkc[i] * 16 + r], acc[i][j]);
    }
  }
}

// Weight gradient  gW[co][k] += sum_n gout[n][co] in[n + d(tap(k))][ci(k)]
// (FP32 atomics).  grid = co_tiles * k_tiles * nsplit blocks of one wave; each
// wave reduces over its voxel range in chunks of 16 (4 voxels per lane group).
__global__ __launch_bounds__(64) void k_conv_wgrad(const uint16_t* __restrict__ in, Dims dm, int cs_in, int ks,
                                                   const uint16_t* __restrict__ gout, int cs_g, int cout, int kp,
                                                   float* __restrict__ gW, int nsplit, long long chunk) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int ncot = (cout + 15) >> 4;
  const int tile = blockIdx.x / nsplit, split = blockIdx.x - (blockIdx.x / nsplit) * nsplit;
  const int tc = tile % ncot, kc = tile / ncot;
  const long long N = dm.n();
  const long long v0 = (long long)split * chunk;
  const long long v1 = v0 + chunk < N ? v0 + chunk : N;
  const int co = tc * 16 + r;
  const int k = kc * 16 + r;
  const int tap = k / cs_in, ci = k - (k / cs_in) * cs_in;
  const bool kvalid = tap < ks * ks * ks;
  int dx = 0, dy = 0, dz = 0;
  if (kvalid) tap_offset(tap, ks, dx, dy, dz);
  f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
  // the 4 voxels of this lane group in the 16-voxel chunk at nb (zero past v1)
  auto slices = [&](long long nb, s4v& a, s4v& b) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long n = nb + 4 * g + j;
      uint16_t av = 0, bv = 0;
      if (n < v1) {
        if (co < cout) av = gout[n * cs_g + co];
        if (kvalid) {
          int x, y, z;
          dm.decode(n, x, y, z);
          const int xx = x + dx, yy = y + dy, zz = z + dz;
          if (dm.inside(xx, yy, zz)) bv = in[dm.encode(xx, yy, zz) * cs_in + ci];
        }
      }
      a[j] = (short)av;
      b[j] = (short)bv;
    }
  };
  // two chunks per instruction (the second may be empty); the loads of U instructions are
  // issued before their MFMAs, which run in the same order as one at a time
  constexpr int U = 4;
  for (long long nb = v0; nb < v1; nb += 32 * U) {
    s4v a0[U], b0[U], a1[U], b1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      slices(nb + 32 * u, a0[u], b0[u]);
      slices(nb + 32 * u + 16, a1[u], b1[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = mfma2(a0[u], a1[u], b0[u], b1[u], acc);
  }
  // D[row = co 4g+j][col = k r]
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int cor = tc * 16 + 4 * g + j;
    if (cor < cout && k < kp && acc[j] != 0.f) atomicAdd(&gW[(long long)cor * kp + k], acc[j]);
  }
}

// Bias gradient gb[co] += sum_n g[n][co] (cs_g <= 256), 256 threads per block.
__global__ void k_bias_grad(const uint16_t* __restrict__ gout, long long N, int cs_g, int cout, float* __restrict__ gb) {
  // items (voxel, group of 4 channels) in memory order, 8-byte loads; the grid's thread
  // count is a multiple of cs_g / 4, so each thread always meets the same channel group
  __shared__ float bins[256];
  const int cq = cs_g >> 2;
  const long long nitem = N * cq;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (int c = threadIdx.x; c < cs_g; c += blockDim.x) bins[c] = 0.f;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (long long i = i0; i < nitem; i += stride) {
    const s4v v = *reinterpret_cast<const s4v*>(gout + 4 * i);
    acc.x += bf2f((uint16_t)v[0]); acc.y += bf2f((uint16_t)v[1]);
    acc.z += bf2f((uint16_t)v[2]); acc.w += bf2f((uint16_t)v[3]);
  }
  __syncthreads();
  const int c4 = (int)(i0 % cq);
  atomicAdd(&bins[4 * c4 + 0], acc.x);
  atomicAdd(&bins[4 * c4 + 1], acc.y);
  atomicAdd(&bins[4 * c4 + 2], acc.z);
  atomicAdd(&bins[4 * c4 + 3], acc.w);
  __syncthreads();
  for (int c = threadIdx.x; c < cout; c += blockDim.x) atomicAdd(&gb[c], bins[c]);
}

// FP32 channel-major volumes [C][src] / scale -> BF16 channels-last [N][cs] (crop
// window (o, dst) of the source; channels C..cs-1 zero).
__global__ void k_to_bf16_crop(const float* __restrict__ x, int C, Dims src, int ox, int oy, int oz, Dims dst,
                               const double* __restrict__ scale, int cs, uint16_t* __restrict__ out) {
  const long long N = dst.n(), ns = src.n();
  const float inv = (float)(1.0 / *scale);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    int x0, y0, z0;
    dst.decode(i, x0, y0, z0);
    const long long j = src.encode(x0 + ox, y0 + oy, z0 + oz);
    for (int c4 = 0; c4 < cs; c4 += 4) {   // cs is a multiple of 4: 8-byte stores
      s4v v;
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = (short)(c4 + q < C ? f2bf(x[(c4 + q) * ns + j] * inv) : (uint16_t)0);
      *reinterpret_cast<s4v*>(out + i * cs + c4) = v;
    }
  }
}

// 2x2x2 average pooling (channels-last).
__global__ void k_avgpool(const uint16_t* __restrict__ in, Dims di, int cs, uint16_t* __restrict__ out, Dims dout) {
  const long long N = dout.n() * cs;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const long long n = i / cs;
    const int c = (int)(i - n * cs);
    int x, y, z;
    dout.decode(n, x, y, z);
    float s = 0.f;
    for (int q = 0; q < 8; ++q) s += bf2f(in[di.encode(2 * x + (q >> 2), 2 * y + ((q >> 1) & 1), 2 * z + (q & 1)) * cs + c]);
    out[i] = f2bf(0.125f * s);
  }
}

// gin[child] = gout[parent]/8 added to gin (average-pool backward).
__global__ void k_avgpool_bwd_add(const uint16_t* __restrict__ gout, Dims dout, int cs, uint16_t* __restrict__ gin, Dims di) {
  const long long N = di.n() * cs;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const long long n = i / cs;
    const int c = (int)(i - n * cs);
    int x, y, z;
    di.decode(n, x, y, z);
    const float v = bf2f(gout[dout.encode(x >> 1, y >> 1, z >> 1) * cs + c]);
    gin[i] = f2bf(bf2f(gin[i]) + 0.125f * v);
  }
}

// out[n] = [skip[n][0:c1], coarse[n/2][0:c2], 0...] (nearest upsampling + concat).
// One thread per (fine voxel, group of 4 channels), 8-byte stores in memory order; a
// group that lies within one source at a 4-aligned offset is one 8-byte load (the
// channel strides are multiples of 4), any other group is gathered channel by channel.
__global__ void k_upcat(const uint16_t* __restrict__ skip, int cs1, int c1, const uint16_t* __restrict__ coarse, int cs2,
                        int c2, Dims df, Dims dc, int cs, uint16_t* __restrict__ out) {
  const int cq = cs >> 2;
  const long long N = df.n() * cq;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const long long n = i / cq;
    const int c = 4 * (int)(i - n * cq);
    int x, y, z;
    df.decode(n, x, y, z);
    const uint16_t* sr = skip + n * cs1;
    const uint16_t* cr = coarse + dc.encode(x >> 1, y >> 1, z >> 1) * cs2;
    s4v v = s4v{0, 0, 0, 0};
    if (c + 4 <= c1) {
      v = *reinterpret_cast<const s4v*>(sr + c);
    } else if (c >= c1 && c + 4 <= c1 + c2 && ((c - c1) & 3) == 0) {
      v = *reinterpret_cast<const s4v*>(cr + (c - c1));
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = c + q;
        v[q] = (short)(cc < c1 ? sr[cc] : (cc < c1 + c2 ? cr[cc - c1] : (uint16_t)0));
      }
    }
    *reinterpret_cast<s4v*>(out + 4 * i) = v;
  }
}

// Backward of k_upcat: gskip[n][c] = g[n][c] (c < c1); gcoarse[m][c] = sum of its 8 children.
__global__ void k_upcat_bwd(const uint16_t* __restrict__ g, int cs, int c1, int c2, Dims df, Dims dc,
                            uint16_t* __restrict__ gskip, int cs1, uint16_t* __restrict__ gcoarse, int cs2) {
  const long long Nf = df.n() * cs1;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < Nf; i += (long long)gridDim.x * blockDim.x) {
    const long long n = i / cs1;
    const int c = (int)(i - n * cs1);
    gskip[i] = c < c1 ? g[n * cs + c] : (uint16_t)0;
  }
  const long long Nc = dc.n() * cs2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < Nc; i += (long long)gridDim.x * blockDim.x) {
    const long long m = i / cs2;
    const int c = (int)(i - m * cs2);
    float s = 0.f;
    if (c < c2) {
      int x, y, z;
      dc.decode(m, x, y, z);
      for (int q = 0; q < 8; ++q) s += bf2f(g[df.encode(2 * x + (q >> 2), 2 * y + ((q >> 1) & 1), 2 * z + (q & 1)) * cs + c1 + c]);
    }
    gcoarse[i] = f2bf(s);
  }
}

// g *= (act > 0)  (ReLU backward, act = the layer's post-ReLU output).
__global__ void k_relu_bwd(uint16_t* __restrict__ g, const uint16_t* __restrict__ act, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    if (!(bf2f(act[i]) > 0.f)) g[i] = 0;
}

// MSE on a crop: loss += sum (y - t/s)^2 / n (FP64 atomics); gy = 2 (y - t/s) / n as BF16 [N][cs].
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, Dims src, int ox, int oy, int oz,
                      Dims dm, const double* __restrict__ scale, int cs, uint16_t* __restrict__ gy, double* __restrict__ loss) {
  __shared__ double part[256];
  const long long N = dm.n();
  const float inv = (float)(1.0 / *scale);
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    int x, yy, z;
    dm.decode(i, x, yy, z);
    const float e = y[i] - t[src.encode(x + ox, yy + oy, z + oz)] * inv;
    acc += (double)e * (double)e;
    gy[i * cs] = f2bf(2.f * e / (float)N);
    for (int c = 1; c < cs; ++c) gy[i * cs + c] = 0;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < (int)blockDim.x; ++q) s += part[q];
    atomicAdd(loss, s / (double)N);
  }
}

// max_i |sum_c x[c][i]| over C channel-major volumes of n voxels: per-block maxima
// folded into *slot with an integer atomic max (the bit patterns of non-negative
// floats order like their values), then k_absmax_final writes it as FP64 to *out
// (1 if the maximum is 0) and clears the slot for the next call.
// Items of 4 consecutive voxels (n is a multiple of 4), channels summed in order.
__global__ void k_absmax(const float* __restrict__ x, long long n, int C, unsigned* __restrict__ slot) {
  __shared__ float part[256];
  float m = 0.f;
  const long long n4 = n >> 2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n4; i += (long long)gridDim.x * blockDim.x) {
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int c = 0; c < C; ++c) {
      const float4 a = reinterpret_cast<const float4*>(x + c * n)[i];
      v.x += a.x; v.y += a.y; v.z += a.z; v.w += a.w;
    }
    m = fmaxf(fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y))), fmaxf(fabsf(v.z), fabsf(v.w)));
  }
  part[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) part[threadIdx.x] = fmaxf(part[threadIdx.x], part[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(slot, __float_as_uint(part[0]));
}
// 1x1x1 convolution to one FP32 output channel (the head): y[n] = b + sum_c W[c] in[n][c],
// W the first row of the packed BF16 forward matrix, FP32 sums.
__global__ void k_head1(const uint16_t* __restrict__ in, long long N, int cs_in, int cin, const uint16_t* __restrict__ W,
                        const float* __restrict__ bias, float* __restrict__ y) {
  const float b = bias[0];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    float acc = 0.f;
    for (int c4 = 0; c4 < cs_in; c4 += 4) {
      const s4v v = *reinterpret_cast<const s4v*>(in + i * cs_in + c4);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (c4 + q < cin) acc += bf2f((uint16_t)v[q]) * bf2f(W[c4 + q]);
    }
    y[i] = acc + b;
  }
}

__global__ void k_absmax_final(unsigned* __restrict__ slot, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    const float t = __uint_as_float(*slot);
    *out = t > 0.f ? (double)t : 1.0;
    *slot = 0u;
  }
}

// rho = s * max(y, 0)
__global__ void k_scale_relu(const float* __restrict__ y, long long n, const double* __restrict__ scale, float* __restrict__ rho) {
  const float s = (float)*scale;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    rho[i] = s * fmaxf(y[i], 0.f);
}

// One layer's matrices for the packing kernels, and the range of the launch's blocks
// that serve it (every layer in one launch: blocks [b0, b0 + nb) take layer l).
struct PackDesc {
  const float* p;          // the layer's weights in the flat FP32 parameters
  float* gp;               // the layer's weight gradient in the flat FP32 gradient
  uint16_t* Wf;
  uint16_t* Wt;
  const float* gWf;
  int cin, cout, ks, cs_in, cs_out, kp, kpt, rows_f, rows_t;
  int pb0, pnb;            // blocks of k_pack_all
  int ub0, unb;            // blocks of k_unpack_all
};

// Master FP32 layer parameters (flat layout W[co][tap][cin], bias) -> BF16 GEMM
// matrices: forward W[co_pad][kp] with k = tap*cs_in + ci, and the flipped,
// transposed matrix of the data gradient Wt[ci_pad][kpt] with k = tap'*cs_out + co,
// Wt[ci][tap'][co] = W[co][ntap-1-tap'][ci].  All nl layers in one launch.
__global__ void k_pack_all(const PackDesc* __restrict__ ds, int nl) {
  int l = 0;
  while (l + 1 < nl && (int)blockIdx.x >= ds[l + 1].pb0) ++l;
  const PackDesc& d = ds[l];
  const int ntap = d.ks * d.ks * d.ks;
  const long long nf = (long long)d.rows_f * d.kp, nt = (long long)d.rows_t * d.kpt;
  for (long long i = (blockIdx.x - d.pb0) * (long long)blockDim.x + threadIdx.x; i < nf + nt;
       i += (long long)d.pnb * blockDim.x) {
    if (i < nf) {
      const int co = (int)(i / d.kp), k = (int)(i - (long long)co * d.kp);
      const int tap = k / d.cs_in, ci = k - tap * d.cs_in;
      float v = 0.f;
      if (co < d.cout && tap < ntap && ci < d.cin) v = d.p[((long long)co * ntap + tap) * d.cin + ci];
      d.Wf[i] = f2bf(v);
    } else {
      const long long j = i - nf;
      const int ci = (int)(j / d.kpt), k = (int)(j - (long long)ci * d.kpt);
      const int tp = k / d.cs_out, co = k - tp * d.cs_out;
      float v = 0.f;
      if (ci < d.cin && tp < ntap && co < d.cout) v = d.p[((long long)co * ntap + (ntap - 1 - tp)) * d.cin + ci];
      d.Wt[j] = f2bf(v);
    }
  }
}

// Gradient of each padded forward GEMM matrix back to the flat layout, all layers in one launch.
__global__ void k_unpack_all(const PackDesc* __restrict__ ds, int nl) {
  int l = 0;
  while (l + 1 < nl && (int)blockIdx.x >= ds[l + 1].ub0) ++l;
  const PackDesc& d = ds[l];
  const int ntap = d.ks * d.ks * d.ks;
  const long long n = (long long)d.cout * ntap * d.cin;
  for (long long i = (blockIdx.x - d.ub0) * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)d.unb * blockDim.x) {
    const int ci = (int)(i % d.cin);
    const long long rest = i / d.cin;
    const int tap = (int)(rest % ntap), co = (int)(rest / ntap);
    d.gp[i] = d.gWf[(long long)co * d.kp + tap * d.cs_in + ci];
  }
}

// Adam (Kingma & Ba 2015) on FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_fill_f32(float* __restrict__ p, long long n, float v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double* __restrict__ p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace net
}  // namespace mh3d
