// Host side of the warm-start network and of the on-GPU training-data generator.
// Included by mh3d.hip after the plan definitions (it uses mh3d_plan_s).
#pragma once
#include <map>
#include <tuple>

#include "net_kernels.hpp"

using namespace mh3d::net;

namespace {

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}
int round4(int c) { return (c + 3) & ~3; }
int round16(int c) { return (c + 15) & ~15; }

struct NetLayer {
  int cin, cout, ks;
  int cs_in, cs_out;       // channel strides of the input / output tensors
  int kp, kpt;             // K of the forward / data-gradient GEMMs (multiples of 16)
  int rows_f, rows_t;      // padded rows of the forward / data-gradient matrices
  long long w_off, b_off;  // offsets in the flat FP32 parameter vector
  uint16_t* Wf = nullptr;  // BF16 forward matrix
  uint16_t* Wt = nullptr;  // BF16 flipped transposed matrix
  float* gWf = nullptr;    // FP32 gradient of the forward matrix (a slice of the network's gW)
};

// Activations and gradients of one grid shape.
struct NetWork {
  int lx, ly, lz;
  std::vector<uint16_t*> bufs;
  uint16_t* x0 = nullptr;                 // input [N0][4]
  std::vector<uint16_t*> ea, es, pl;      // enc conv a / conv b (skip) outputs, pooled inputs (level l+1)
  std::vector<uint16_t*> cat, da, db;     // decoder concat input, conv a, conv b outputs
  std::vector<uint16_t*> g1, g2, g3, gs;  // gradient scratch per level (max channel stride) and skip grads
  float* y = nullptr;                     // head output FP32 [N0]
  float* xin = nullptr;                   // warm start: per-harmonic back-projections [C][N0] (lazy)
  uint16_t* gy = nullptr;                 // head output gradient [N0][4]
  double* scale = nullptr;                // max |x| of the current input
  double* loss = nullptr;
};

}  // namespace

struct mh3d_net_s {
  std::vector<int> widths;
  int in_ch = 1;
  std::vector<NetLayer> layers;
  long long nparam = 0;
  float* p = nullptr;        // FP32 master parameters (flat layout of oracle/unet.py)
  float* g = nullptr;        // FP32 gradient, same layout
  float* m = nullptr;        // Adam moments
  float* v = nullptr;
  int64_t step = 0;
  hipStream_t stream;
  std::map<std::tuple<int, int, int>, NetWork> work;
  bool packed = false;
  float* gW = nullptr;           // every layer's FP32 forward-matrix gradient, one buffer
  long long gW_len = 0;
  PackDesc* pack = nullptr;      // device table of the layers for k_pack_all / k_unpack_all
  int pack_blocks = 0, unpack_blocks = 0;
};

namespace {

mh3d_status net_alloc(void** ptr, size_t bytes) {
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    *ptr = nullptr;
    return fail(MH3D_ERR_OOM, "hipMalloc(%zu) failed in the network", bytes);
  }
  return MH3D_OK;
}

int grid_for(long long n, int block = 256) {
  long long b = (n + block - 1) / block;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

// layer order: enc0a enc0b ... enc(L-1)b, dec(L-2)a dec(L-2)b ... dec0a dec0b, head
int enc_index(int l, int ab) { return 2 * l + ab; }
int dec_index(int L, int l, int ab) { return 2 * L + 2 * (L - 2 - l) + ab; }

mh3d_status net_pack(mh3d_net_t n) {
  k_pack_all<<<n->pack_blocks, 256, 0, n->stream>>>(n->pack, (int)n->layers.size());
  CHK(last_launch("k_pack_all"));
  n->packed = true;
  return MH3D_OK;
}

mh3d_status net_work(mh3d_net_t n, int nx, int ny, int nz, NetWork** out) {
  auto key = std::make_tuple(nx, ny, nz);
  auto it = n->work.find(key);
  if (it != n->work.end()) { *out = &it->second; return MH3D_OK; }
  const int L = (int)n->widths.size();
  NetWork w;
  w.lx = ilog2(nx); w.ly = ilog2(ny); w.lz = ilog2(nz);
  auto nvox = [&](int l) { return 1ll << (w.lx + w.ly + w.lz - 3 * l); };
  auto mk = [&](long long elems, uint16_t** p) -> mh3d_status {
    void* q = nullptr;
    CHK(net_alloc(&q, sizeof(uint16_t) * (size_t)elems));
    (void)hipMemsetAsync(q, 0, sizeof(uint16_t) * (size_t)elems, n->stream);
    w.bufs.push_back((uint16_t*)q);
    *p = (uint16_t*)q;
    return MH3D_OK;
  };
  CHK(mk(nvox(0) * round4(n->in_ch), &w.x0));
  w.ea.resize(L); w.es.resize(L); w.pl.resize(L); w.cat.resize(L); w.da.resize(L); w.db.resize(L);
  w.g1.resize(L); w.g2.resize(L); w.g3.resize(L); w.gs.resize(L);
  int cmax_all = 4;
  for (int l = 0; l < L; ++l) {
    const int cs = round4(n->widths[l]);
    const int cats = l < L - 1 ? round4(n->widths[l] + n->widths[l + 1]) : 4;
    const int cmax = std::max(std::max(cs, cats), l ? round4(n->widths[l - 1]) : 4);
    cmax_all = std::max(cmax_all, cmax);
    CHK(mk(nvox(l) * cs, &w.ea[l]));
    CHK(mk(nvox(l) * cs, &w.es[l]));
    if (l) CHK(mk(nvox(l) * round4(n->widths[l - 1]), &w.pl[l]));
    if (l < L - 1) {
      CHK(mk(nvox(l) * cats, &w.cat[l]));
      CHK(mk(nvox(l) * cs, &w.da[l]));
      CHK(mk(nvox(l) * cs, &w.db[l]));
    }
    CHK(mk(nvox(l) * cmax, &w.g1[l]));
    CHK(mk(nvox(l) * cmax, &w.g2[l]));
    CHK(mk(nvox(l) * cmax, &w.g3[l]));
    CHK(mk(nvox(l) * cs, &w.gs[l]));
  }
  CHK(mk(nvox(0) * 4, &w.gy));
  CHK(net_alloc((void**)&w.y, sizeof(float) * (size_t)nvox(0)));
  // [scale, loss, (unused), (unused), absmax slot]
  CHK(net_alloc((void**)&w.scale, sizeof(double) * 5));
  (void)hipMemsetAsync(w.scale, 0, sizeof(double) * 5, n->stream);
  w.loss = w.scale + 1;
  (void)cmax_all;
  auto res = n->work.emplace(key, w);
  *out = &res.first->second;
  return MH3D_OK;
}

Dims dims_of(const NetWork& w, int l) { return Dims{w.lx - l, w.ly - l, w.lz - l}; }

// One convolution out = act(conv(in, W) + bias), BF16 channels-last output with
// channel stride cs_out (or FP32 single-channel for the head).  3x3x3 layers with at
// most 32 output channels on grids of at least 4 x 4 x 16 run the LDS-tiled kernel.
// k_conv_ct for the channel strides it is compiled for (false: none, or kp does not
// match the compile-time K).
template <int CS>
bool conv_ct_try(hipStream_t s, int ntile, bool relu, int blocks, const uint16_t* in, Dims dm, const uint16_t* W,
                 int kp, const float* bias, int cout, int cs_out, uint16_t* o) {
  if (kp != 16 * ((27 * CS + 15) / 16) || ntile < 1 || ntile > 2) return false;
  if (ntile == 1) {
    if (relu) k_conv_ct<CS, 1, true><<<blocks, 256, conv_ct_lds<CS, 1>(), s>>>(in, dm, W, kp, bias, cout, cs_out, o, nullptr);
    else k_conv_ct<CS, 1, false><<<blocks, 256, conv_ct_lds<CS, 1>(), s>>>(in, dm, W, kp, bias, cout, cs_out, o, nullptr);
  } else {
    if (relu) k_conv_ct<CS, 2, true><<<blocks, 256, conv_ct_lds<CS, 2>(), s>>>(in, dm, W, kp, bias, cout, cs_out, o, nullptr);
    else k_conv_ct<CS, 2, false><<<blocks, 256, conv_ct_lds<CS, 2>(), s>>>(in, dm, W, kp, bias, cout, cs_out, o, nullptr);
  }
  return true;
}

// The decoder's first convolution (ReLU) on [skip, upsampled coarse] read in place, for
// the (channel stride, skip channels) pairs compiled here; false otherwise.
template <int CS, int C1>
bool conv_ct_cat_try(hipStream_t s, int ntile, int blocks, const uint16_t* skip, const uint16_t* coarse, Dims dm,
                     const uint16_t* W, int kp, const float* bias, int cout, int cs_out, uint16_t* o) {
  if (kp != 16 * ((27 * CS + 15) / 16) || ntile < 1 || ntile > 2) return false;
  if (ntile == 1)
    k_conv_ct<CS, 1, true, C1><<<blocks, 256, conv_ct_lds<CS, 1>(), s>>>(skip, dm, W, kp, bias, cout, cs_out, o, coarse);
  else
    k_conv_ct<CS, 2, true, C1><<<blocks, 256, conv_ct_lds<CS, 2>(), s>>>(skip, dm, W, kp, bias, cout, cs_out, o, coarse);
  return true;
}

// k_conv_splitk8 with the output tile count as a compile-time constant.
template <int NT>
void splitk8_nt(hipStream_t s, bool relu, int blocks, const uint16_t* in, Dims dm, int cs_in, int ks, const uint16_t* W,
                int kp, const float* bias, int cout, int cs_out, uint16_t* o) {
  if (relu) k_conv_splitk8<true, NT><<<blocks, 256, 0, s>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o);
  else k_conv_splitk8<false, NT><<<blocks, 256, 0, s>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o);
}

void splitk8(hipStream_t s, bool relu, int ntile, int blocks, const uint16_t* in, Dims dm, int cs_in, int ks,
             const uint16_t* W, int kp, const float* bias, int cout, int cs_out, uint16_t* o) {
  switch (ntile) {
    case 1: splitk8_nt<1>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    case 2: splitk8_nt<2>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    case 3: splitk8_nt<3>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    case 4: splitk8_nt<4>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    case 5: splitk8_nt<5>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    case 6: splitk8_nt<6>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    case 7: splitk8_nt<7>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
    default: splitk8_nt<8>(s, relu, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o); break;
  }
}

bool conv_ct(hipStream_t s, int cs_in, int ntile, bool relu, int blocks, const uint16_t* in, Dims dm, const uint16_t* W,
             int kp, const float* bias, int cout, int cs_out, uint16_t* o) {
  switch (cs_in) {
    case 4: return conv_ct_try<4>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    case 8: return conv_ct_try<8>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    case 12: return conv_ct_try<12>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    case 16: return conv_ct_try<16>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    case 24: return conv_ct_try<24>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    case 32: return conv_ct_try<32>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    case 48: return conv_ct_try<48>(s, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o);
    default: return false;
  }
}

mh3d_status launch_conv(mh3d_net_t n, const uint16_t* in, Dims dm, int cs_in, int ks, const uint16_t* W, int kp,
                        const float* bias, int cout, int cs_out, void* out, bool relu, bool f32) {
  const long long N = 1ll << (dm.lx + dm.ly + dm.lz);
  const int ntile = (cout + 15) / 16;
  const size_t halo = sizeof(uint16_t) * 648 * (size_t)cs_in;
  if (!f32 && ks == 3 && ntile <= 2 && dm.lz >= 4 && dm.ly >= 2 && dm.lx >= 2 && halo <= 64 * 1024) {
    const int blocks = (int)(N / 256);
    uint16_t* o = reinterpret_cast<uint16_t*>(out);
    if (conv_ct(n->stream, cs_in, ntile, relu, blocks, in, dm, W, kp, bias, cout, cs_out, o))
      return last_launch("k_conv_ct");
    if (relu) {
      if (ntile == 1) k_conv_tiled<true, 1><<<blocks, 256, halo, n->stream>>>(in, dm, cs_in, W, kp, bias, cout, cs_out, o);
      else k_conv_tiled<true, 2><<<blocks, 256, halo, n->stream>>>(in, dm, cs_in, W, kp, bias, cout, cs_out, o);
    } else {
      if (ntile == 1) k_conv_tiled<false, 1><<<blocks, 256, halo, n->stream>>>(in, dm, cs_in, W, kp, bias, cout, cs_out, o);
      else k_conv_tiled<false, 2><<<blocks, 256, halo, n->stream>>>(in, dm, cs_in, W, kp, bias, cout, cs_out, o);
    }
    return last_launch("k_conv_tiled");
  }
  if (!f32 && (kp >> 4) >= 32 && N <= (1ll << 17)) {
    // deep reduction on a small grid: split K over the block's waves
    const int blocks = (int)((N + 15) / 16);
    uint16_t* o = reinterpret_cast<uint16_t*>(out);
    if (cs_in % 8 == 0 && ntile <= 8) {
      splitk8(n->stream, relu, ntile, blocks, in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o);
      return last_launch("k_conv_splitk8");
    }
    if (relu) k_conv_splitk<true><<<blocks, 256, 0, n->stream>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o);
    else k_conv_splitk<false><<<blocks, 256, 0, n->stream>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, o);
    return last_launch("k_conv_splitk");
  }
  if (f32 && ks == 1 && cout == 1) {   // the head: one output channel
    k_head1<<<std::min(grid_for(N, 256), 8192), 256, 0, n->stream>>>(in, N, cs_in, cs_in, W, bias,
                                                                   reinterpret_cast<float*>(out));
    return last_launch("k_head1");
  }
  const int blocks = (int)((N + 63) / 64);
  if (f32) k_conv<false, true><<<blocks, 256, 0, n->stream>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, out);
  else if (relu) k_conv<true, false><<<blocks, 256, 0, n->stream>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, out);
  else k_conv<false, false><<<blocks, 256, 0, n->stream>>>(in, dm, cs_in, ks, W, kp, bias, cout, cs_out, out);
  return last_launch("k_conv");
}

mh3d_status conv_fwd(mh3d_net_t n, const NetLayer& ly, const uint16_t* in, Dims dm, void* out, bool relu, bool f32) {
  return launch_conv(n, in, dm, ly.cs_in, ly.ks, ly.Wf, ly.kp, n->p + ly.b_off, ly.cout, ly.cs_out, out, relu, f32);
}

// The decoder's first convolution with ReLU on the concatenation of skip (c1 channels,
// stride c1) and the coarse tensor upsampled by 2 (c2 channels, stride c2), read in
// place where k_conv_ct is compiled for it (c1 + c2 a compiled stride, no padding
// channels); false: the caller concatenates first.
bool conv_fwd_cat(mh3d_net_t n, const NetLayer& ly, const uint16_t* skip, int c1, const uint16_t* coarse, int c2, Dims dm,
                  uint16_t* out) {
  const int ntile = (ly.cout + 15) / 16;
  if (ly.ks != 3 || c1 % 4 || c2 % 4 || ly.cs_in != c1 + c2 || ntile > 2 || dm.lz < 4 || dm.ly < 2 || dm.lx < 2)
    return false;
  const int blocks = (int)((1ll << (dm.lx + dm.ly + dm.lz)) / 256);
  const float* bias = n->p + ly.b_off;
  bool ok = false;
  if (c1 == 4 && c2 == 8) ok = conv_ct_cat_try<12, 4>(n->stream, ntile, blocks, skip, coarse, dm, ly.Wf, ly.kp, bias, ly.cout, ly.cs_out, out);
  else if (c1 == 8 && c2 == 16) ok = conv_ct_cat_try<24, 8>(n->stream, ntile, blocks, skip, coarse, dm, ly.Wf, ly.kp, bias, ly.cout, ly.cs_out, out);
  else if (c1 == 16 && c2 == 32) ok = conv_ct_cat_try<48, 16>(n->stream, ntile, blocks, skip, coarse, dm, ly.Wf, ly.kp, bias, ly.cout, ly.cs_out, out);
  return ok;
}

// Gradients of one conv layer given the gradient g of its (pre-activation) output:
// accumulates dW, db and writes the input gradient gin (unless null).
mh3d_status conv_bwd(mh3d_net_t n, const NetLayer& ly, const uint16_t* in, Dims dm, const uint16_t* g, int cs_g,
                     uint16_t* gin, float* zero_bias) {
  const long long N = 1ll << (dm.lx + dm.ly + dm.lz);
  const int ncot = (ly.cout + 15) / 16, nkc = ly.kp / 16;
  const size_t wlds = sizeof(uint16_t) * (648 * (size_t)ly.cs_in + 256 * 16 * (size_t)ncot);
  if (ly.ks == 3 && dm.lz >= 4 && dm.ly >= 2 && dm.lx >= 2 && wlds <= 96 * 1024) {
    const int ntiles = (int)(N >> 8);
    const int nbg = (ncot * nkc + 15) / 16;
    int tpb = (int)((ntiles * (long long)nbg + 767) / 768);
    tpb = std::max(1, std::min(tpb, 64));
    const dim3 grid((ntiles + tpb - 1) / tpb, nbg);
    k_conv_wgrad_tiled<<<grid, 256, wlds, n->stream>>>(in, dm, ly.cs_in, g, cs_g, ly.cout, ly.kp, ly.gWf, tpb);
    CHK(last_launch("k_conv_wgrad_tiled"));
  } else {
    // voxel ranges of 256 per wave (8 MFMA instructions): enough waves in flight on the
    // small grids and the 1x1x1 head, whose chains are their loads' latency
    long long chunk = 256;
    int nsplit = (int)((N + chunk - 1) / chunk);
    k_conv_wgrad<<<ncot * nkc * nsplit, 64, 0, n->stream>>>(in, dm, ly.cs_in, ly.ks, g, cs_g, ly.cout, ly.kp, ly.gWf,
                                                            nsplit, chunk);
    CHK(last_launch("k_conv_wgrad"));
  }
  {
    // cs_g <= 256 channels; blocks: a multiple of cs_g / 4 (each thread keeps one channel group)
    if (cs_g > 256 || cs_g % 4) return fail(MH3D_ERR_UNSUPPORTED, "gradient channel stride %d (at most 256)", cs_g);
    const int cq = cs_g / 4;
    const long long items = N * cq;
    long long nb = std::max<long long>(1, std::min<long long>(items / (256 * 16), 1024 / cq));
    k_bias_grad<<<(int)(nb * cq), 256, 0, n->stream>>>(g, N, cs_g, ly.cout, n->g + ly.b_off);
  }
  CHK(last_launch("k_bias_grad"));
  if (gin) {
    // data gradient = convolution of g with the flipped, transposed weights (no bias)
    CHK(launch_conv(n, g, dm, cs_g, ly.ks, ly.Wt, ly.kpt, zero_bias, ly.cin, ly.cs_in, gin, false, false));
  }
  return MH3D_OK;
}

// x (FP32, volume grid `src`, crop window o + dst dims) -> forward through the net;
// result FP32 in w->y.  Scale s = max |x| over the whole source volume.
mh3d_status net_forward(mh3d_net_t n, NetWork* w, const float* x, Dims src, long long nsrc, int ox, int oy, int oz,
                        bool infer = false) {
  const int L = (int)n->widths.size();
  if (!n->packed) CHK(net_pack(n));
  unsigned* slot = reinterpret_cast<unsigned*>(w->scale + 4);
  if (nsrc % 4) return fail(MH3D_ERR_INVALID, "volume size %lld is not a multiple of 4", nsrc);
  k_absmax<<<std::min(grid_for(nsrc / 4, 256), 4096), 256, 0, n->stream>>>(x, nsrc, n->in_ch, slot);
  CHK(last_launch("k_absmax"));
  k_absmax_final<<<1, 64, 0, n->stream>>>(slot, w->scale);
  CHK(last_launch("k_absmax_final"));
  Dims d0 = dims_of(*w, 0);
  k_to_bf16_crop<<<grid_for(d0.n()), 256, 0, n->stream>>>(x, n->in_ch, src, ox, oy, oz, d0, w->scale,
                                                          round4(n->in_ch), w->x0);
  CHK(last_launch("k_to_bf16_crop"));
  const uint16_t* h = w->x0;
  for (int l = 0; l < L; ++l) {
    Dims dl = dims_of(*w, l);
    if (l) {
      const int cs = round4(n->widths[l - 1]);
      k_avgpool<<<grid_for(dl.n() * cs), 256, 0, n->stream>>>(h, dims_of(*w, l - 1), cs, w->pl[l], dl);
      CHK(last_launch("k_avgpool"));
      h = w->pl[l];
    }
    CHK(conv_fwd(n, n->layers[enc_index(l, 0)], h, dl, w->ea[l], true, false));
    CHK(conv_fwd(n, n->layers[enc_index(l, 1)], w->ea[l], dl, w->es[l], true, false));
    h = w->es[l];
  }
  for (int l = L - 2; l >= 0; --l) {
    Dims dl = dims_of(*w, l);
    const int c1 = n->widths[l], c2 = n->widths[l + 1];
    const int cats = round4(c1 + c2);
    const NetLayer& la = n->layers[dec_index(L, l, 0)];
    // inference reads the concatenation in place where it can (training keeps the
    // concatenated tensor: the weight gradient reads it)
    if (infer && conv_fwd_cat(n, la, w->es[l], c1, h, c2, dl, w->da[l])) {
      CHK(last_launch("k_conv_ct (concatenation read in place)"));
    } else {
      k_upcat<<<grid_for(dl.n() * (cats / 4)), 256, 0, n->stream>>>(w->es[l], round4(c1), c1, h, round4(c2), c2, dl,
                                                              dims_of(*w, l + 1), cats, w->cat[l]);
      CHK(last_launch("k_upcat"));
      CHK(conv_fwd(n, la, w->cat[l], dl, w->da[l], true, false));
    }
    CHK(conv_fwd(n, n->layers[dec_index(L, l, 1)], w->da[l], dl, w->db[l], true, false));
    h = w->db[l];
  }
  CHK(conv_fwd(n, n->layers.back(), h, d0, w->y, false, true));
  return MH3D_OK;
}

mh3d_status net_backward(mh3d_net_t n, NetWork* w) {
  const int L = (int)n->widths.size();
  float* zb = n->g + n->nparam;   // zero bias of the data-gradient convolutions (tail of the gradient buffer)
  Dims d0 = dims_of(*w, 0);
  // head (1x1x1): gradient of the last decoder output
  const uint16_t* top = L >= 2 ? w->db[0] : w->es[0];
  uint16_t* g = w->g1[0];
  CHK(conv_bwd(n, n->layers.back(), top, d0, w->gy, 4, g, zb));
  // decoder, level 0 upwards: g is the gradient of db[l] (post-ReLU output)
  for (int l = 0; l <= L - 2; ++l) {
    Dims dl = dims_of(*w, l);
    const int cs = round4(n->widths[l]);
    const NetLayer& lb = n->layers[dec_index(L, l, 1)];
    const NetLayer& la = n->layers[dec_index(L, l, 0)];
    k_relu_bwd<<<grid_for(dl.n() * cs), 256, 0, n->stream>>>(g, w->db[l], dl.n() * cs);
    CHK(last_launch("k_relu_bwd"));
    uint16_t* g_da = (g == w->g1[l]) ? w->g2[l] : w->g1[l];
    CHK(conv_bwd(n, lb, w->da[l], dl, g, cs, g_da, zb));
    k_relu_bwd<<<grid_for(dl.n() * cs), 256, 0, n->stream>>>(g_da, w->da[l], dl.n() * cs);
    CHK(last_launch("k_relu_bwd"));
    const int cats = round4(n->widths[l] + n->widths[l + 1]);
    uint16_t* g_cat = w->g3[l];
    CHK(conv_bwd(n, la, w->cat[l], dl, g_da, cs, g_cat, zb));
    // split: skip part -> gs[l], coarse part -> gradient of the next level's output
    Dims dc = dims_of(*w, l + 1);
    const int cs2 = round4(n->widths[l + 1]);
    uint16_t* g_next = w->g1[l + 1];
    k_upcat_bwd<<<grid_for(dl.n() * cs), 256, 0, n->stream>>>(g_cat, cats, n->widths[l], n->widths[l + 1], dl, dc,
                                                              w->gs[l], cs, g_next, cs2);
    CHK(last_launch("k_upcat_bwd"));
    g = g_next;
  }
  // encoder, bottom level downwards: g is the gradient of es[l]
  for (int l = L - 1; l >= 0; --l) {
    Dims dl = dims_of(*w, l);
    const int cs = round4(n->widths[l]);
    if (l < L - 1) {
      // total gradient of the skip tensor: concat part (gs) + pooled part (already in g)
      // g currently holds the pooled-path gradient accumulated into gs[l]
      g = w->gs[l];
    }
    const NetLayer& lb = n->layers[enc_index(l, 1)];
    const NetLayer& la = n->layers[enc_index(l, 0)];
    k_relu_bwd<<<grid_for(dl.n() * cs), 256, 0, n->stream>>>(g, w->es[l], dl.n() * cs);
    CHK(last_launch("k_relu_bwd"));
    uint16_t* g_ea = (g == w->g2[l]) ? w->g3[l] : w->g2[l];
    CHK(conv_bwd(n, lb, w->ea[l], dl, g, cs, g_ea, zb));
    k_relu_bwd<<<grid_for(dl.n() * cs), 256, 0, n->stream>>>(g_ea, w->ea[l], dl.n() * cs);
    CHK(last_launch("k_relu_bwd"));
    const uint16_t* in = l ? w->pl[l] : w->x0;
    if (l) {
      uint16_t* g_in = (g_ea == w->g1[l]) ? w->g3[l] : w->g1[l];
      CHK(conv_bwd(n, la, in, dl, g_ea, cs, g_in, zb));
      // average-pool backward adds into the skip gradient of level l-1
      const int csp = round4(n->widths[l - 1]);
      k_avgpool_bwd_add<<<grid_for(dims_of(*w, l - 1).n() * csp), 256, 0, n->stream>>>(g_in, dl, csp, w->gs[l - 1],
                                                                                       dims_of(*w, l - 1));
      CHK(last_launch("k_avgpool_bwd_add"));
    } else {
      CHK(conv_bwd(n, la, in, dl, g_ea, cs, nullptr, zb));
    }
  }
  // padded forward-matrix gradients -> flat layout
  k_unpack_all<<<n->unpack_blocks, 256, 0, n->stream>>>(n->pack, (int)n->layers.size());
  CHK(last_launch("k_unpack_all"));
  return MH3D_OK;
}

mh3d_status net_zero_grads(mh3d_net_t n) {
  k_fill_f32<<<grid_for(n->nparam), 256, 0, n->stream>>>(n->g, n->nparam + 128, 0.f);
  CHK(last_launch("k_fill_f32"));
  k_fill_f32<<<grid_for(n->gW_len), 256, 0, n->stream>>>(n->gW, n->gW_len, 0.f);
  CHK(last_launch("k_fill_f32"));
  return MH3D_OK;
}

// He-normal initialisation from Philox (Box-Muller), zero biases.
__global__ void k_net_init(float* __restrict__ p, long long wo, long long nw, int fan_in, uint64_t seed, uint32_t stream) {
  const float sd = sqrtf(2.f / (float)fan_in);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nw; i += (long long)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)i, stream, 0u, 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const float u1 = ((float)c[0] + 0.5f) * 2.3283064365386963e-10f;
    const float u2 = ((float)c[1] + 0.5f) * 2.3283064365386963e-10f;
    p[wo + i] = sd * sqrtf(-2.f * logf(u1)) * cospif(2.f * u2);
  }
}

}  // namespace

// ============================================================================ network ABI
extern "C" mh3d_status mh3d_net_create(int32_t levels, const int32_t* widths, int32_t in_channels, uint64_t seed,
                                       void* stream, mh3d_net_t* out) {
  if (!out) return fail(MH3D_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (levels < 2 || levels > 6 || !widths) return fail(MH3D_ERR_INVALID, "levels must be in [2, 6]");
  if (in_channels < 1 || in_channels > 32) return fail(MH3D_ERR_INVALID, "in_channels must be in [1, 32]");
  for (int l = 0; l < levels; ++l)
    if (widths[l] < 1 || widths[l] > 16 * NT_MAX) return fail(MH3D_ERR_INVALID, "width %d out of range", widths[l]);
  // the data gradient of a decoder's first convolution has widths[l] + widths[l+1]
  // output channels, which must fit one wave's tiles (and the zero-bias tail)
  for (int l = 0; l + 1 < levels; ++l)
    if (widths[l] + widths[l + 1] > 16 * NT_MAX) return fail(MH3D_ERR_INVALID, "concat width too large");
  mh3d_net_t n = new mh3d_net_s();
  n->widths.assign(widths, widths + levels);
  n->in_ch = in_channels;
  n->stream = reinterpret_cast<hipStream_t>(stream);
  const int L = levels;
  // layer list in the flat parameter order
  struct Spec { int cin, cout, ks; };
  std::vector<Spec> specs;
  int cin = in_channels;
  for (int l = 0; l < L; ++l) {
    specs.push_back({cin, widths[l], 3});
    specs.push_back({widths[l], widths[l], 3});
    cin = widths[l];
  }
  for (int l = L - 2; l >= 0; --l) {
    specs.push_back({widths[l] + widths[l + 1], widths[l], 3});
    specs.push_back({widths[l], widths[l], 3});
  }
  specs.push_back({widths[0], 1, 1});
  long long off = 0;
  for (const Spec& s : specs) {
    NetLayer ly;
    ly.cin = s.cin;
    ly.cout = s.cout;
    ly.ks = s.ks;
    ly.cs_in = round4(s.cin);
    ly.cs_out = round4(s.cout);
    const int ntap = s.ks * s.ks * s.ks;
    ly.kp = round16(ntap * ly.cs_in);
    ly.kpt = round16(ntap * ly.cs_out);
    ly.rows_f = round16(s.cout);
    ly.rows_t = round16(s.cin);
    ly.w_off = off;
    off += (long long)s.cout * ntap * s.cin;
    ly.b_off = off;
    off += s.cout;
    n->layers.push_back(ly);
  }
  n->nparam = off;
  auto bail = [&](mh3d_status st) { mh3d_net_destroy(n); return st; };
  mh3d_status st;
  if ((st = net_alloc((void**)&n->p, sizeof(float) * (off + 128))) != MH3D_OK) return bail(st);
  if ((st = net_alloc((void**)&n->g, sizeof(float) * (off + 128))) != MH3D_OK) return bail(st);
  if ((st = net_alloc((void**)&n->m, sizeof(float) * off)) != MH3D_OK) return bail(st);
  if ((st = net_alloc((void**)&n->v, sizeof(float) * off)) != MH3D_OK) return bail(st);
  for (auto& ly : n->layers) {
    if ((st = net_alloc((void**)&ly.Wf, sizeof(uint16_t) * (size_t)ly.rows_f * ly.kp)) != MH3D_OK) return bail(st);
    if ((st = net_alloc((void**)&ly.Wt, sizeof(uint16_t) * (size_t)ly.rows_t * ly.kpt)) != MH3D_OK) return bail(st);
    n->gW_len += ((long long)ly.rows_f * ly.kp + 63) & ~63ll;   // 256-byte aligned slices
  }
  if ((st = net_alloc((void**)&n->gW, sizeof(float) * (size_t)n->gW_len)) != MH3D_OK) return bail(st);
  {
    // the layer table of the one-launch packing kernels (blocks per layer as one
    // launch per layer would take, at most 1024)
    std::vector<PackDesc> pd(n->layers.size());
    long long goff = 0;
    for (size_t i = 0; i < n->layers.size(); ++i) {
      NetLayer& ly = n->layers[i];
      ly.gWf = n->gW + goff;
      goff += ((long long)ly.rows_f * ly.kp + 63) & ~63ll;
      PackDesc& d = pd[i];
      d.p = n->p + ly.w_off;
      d.gp = n->g + ly.w_off;
      d.Wf = ly.Wf;
      d.Wt = ly.Wt;
      d.gWf = ly.gWf;
      d.cin = ly.cin; d.cout = ly.cout; d.ks = ly.ks; d.cs_in = ly.cs_in; d.cs_out = ly.cs_out;
      d.kp = ly.kp; d.kpt = ly.kpt; d.rows_f = ly.rows_f; d.rows_t = ly.rows_t;
      d.pb0 = n->pack_blocks;
      d.pnb = std::min(grid_for((long long)ly.rows_f * ly.kp + (long long)ly.rows_t * ly.kpt), 1024);
      n->pack_blocks += d.pnb;
      d.ub0 = n->unpack_blocks;
      d.unb = std::min(grid_for((long long)ly.cout * ly.ks * ly.ks * ly.ks * ly.cin), 1024);
      n->unpack_blocks += d.unb;
    }
    if ((st = net_alloc((void**)&n->pack, sizeof(PackDesc) * pd.size())) != MH3D_OK) return bail(st);
    if (hipMemcpy(n->pack, pd.data(), sizeof(PackDesc) * pd.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(MH3D_ERR_HIP, "network layer table upload failed"));
  }
  k_fill_f32<<<grid_for(off + 128), 256, 0, n->stream>>>(n->p, off + 128, 0.f);
  k_fill_f32<<<grid_for(off), 256, 0, n->stream>>>(n->m, off, 0.f);
  k_fill_f32<<<grid_for(off), 256, 0, n->stream>>>(n->v, off, 0.f);
  for (size_t i = 0; i < n->layers.size(); ++i) {
    const NetLayer& ly = n->layers[i];
    const long long nw = (long long)ly.cout * ly.ks * ly.ks * ly.ks * ly.cin;
    k_net_init<<<grid_for(nw), 256, 0, n->stream>>>(n->p, ly.w_off, nw, ly.cin * ly.ks * ly.ks * ly.ks, seed, (uint32_t)i);
  }
  if ((st = last_launch("k_net_init")) != MH3D_OK) return bail(st);
  if ((st = net_zero_grads(n)) != MH3D_OK) return bail(st);
  if (hipStreamSynchronize(n->stream) != hipSuccess) return bail(fail(MH3D_ERR_HIP, "network init failed"));
  *out = n;
  return MH3D_OK;
}

extern "C" void mh3d_net_destroy(mh3d_net_t n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  for (auto& kv : n->work) {
    for (auto* b : kv.second.bufs) (void)hipFree(b);
    if (kv.second.y) (void)hipFree(kv.second.y);
    if (kv.second.scale) (void)hipFree(kv.second.scale);
    if (kv.second.xin) (void)hipFree(kv.second.xin);
  }
  for (auto& ly : n->layers) {
    if (ly.Wf) (void)hipFree(ly.Wf);
    if (ly.Wt) (void)hipFree(ly.Wt);
  }
  void* bufs[] = {n->p, n->g, n->m, n->v, n->gW, n->pack};
  for (void* q : bufs)
    if (q) (void)hipFree(q);
  delete n;
}

extern "C" int64_t mh3d_net_param_count(mh3d_net_t n) { return n ? n->nparam : 0; }

extern "C" mh3d_status mh3d_net_params(mh3d_net_t n, float* dst, int32_t set) {
  if (!n || !dst) return fail(MH3D_ERR_INVALID, "NULL argument");
  if (set) {
    HIPCHK(hipMemcpyAsync(n->p, dst, sizeof(float) * n->nparam, hipMemcpyDeviceToDevice, n->stream));
    n->packed = false;
  } else {
    HIPCHK(hipMemcpyAsync(dst, n->p, sizeof(float) * n->nparam, hipMemcpyDeviceToDevice, n->stream));
  }
  HIPCHK(hipStreamSynchronize(n->stream));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_net_grads(mh3d_net_t n, float* dst) {
  if (!n || !dst) return fail(MH3D_ERR_INVALID, "NULL argument");
  HIPCHK(hipMemcpyAsync(dst, n->g, sizeof(float) * n->nparam, hipMemcpyDeviceToDevice, n->stream));
  HIPCHK(hipStreamSynchronize(n->stream));
  return MH3D_OK;
}

static mh3d_status net_check_dims(mh3d_net_t n, int nx, int ny, int nz) {
  const int L = (int)n->widths.size();
  const int dims[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a)
    if (ilog2(dims[a]) < 0 || dims[a] < (1 << L)) return fail(MH3D_ERR_INVALID, "network grids must be powers of two >= 2^levels");
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_net_forward(mh3d_net_t n, const float* x, int32_t nx, int32_t ny, int32_t nz, float* y) {
  if (!n || !x || !y) return fail(MH3D_ERR_INVALID, "NULL argument");
  CHK(net_check_dims(n, nx, ny, nz));
  NetWork* w;
  CHK(net_work(n, nx, ny, nz, &w));
  Dims src{ilog2(nx), ilog2(ny), ilog2(nz)};
  CHK(net_forward(n, w, x, src, (long long)nx * ny * nz, 0, 0, 0, true));
  HIPCHK(hipMemcpyAsync(y, w->y, sizeof(float) * (size_t)nx * ny * nz, hipMemcpyDeviceToDevice, n->stream));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_net_loss_grad(mh3d_net_t n, const float* x, const float* t, int32_t nx, int32_t ny,
                                          int32_t nz, const int32_t* crop, double* loss) {
  if (!n || !x || !t) return fail(MH3D_ERR_INVALID, "NULL argument");
  CHK(net_check_dims(n, nx, ny, nz));
  int o[3] = {0, 0, 0}, c[3] = {nx, ny, nz};
  if (crop) {
    for (int a = 0; a < 3; ++a) { o[a] = crop[a]; c[a] = crop[3 + a]; }
    const int full[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a)
      if (o[a] < 0 || c[a] < 1 || o[a] + c[a] > full[a]) return fail(MH3D_ERR_INVALID, "crop outside the volume");
    CHK(net_check_dims(n, c[0], c[1], c[2]));
  }
  NetWork* w;
  CHK(net_work(n, c[0], c[1], c[2], &w));
  Dims src{ilog2(nx), ilog2(ny), ilog2(nz)};
  CHK(net_zero_grads(n));
  CHK(net_forward(n, w, x, src, (long long)nx * ny * nz, o[0], o[1], o[2]));
  Dims d0 = dims_of(*w, 0);
  k_fill_f64<<<1, 64, 0, n->stream>>>(w->loss, 1, 0.0);
  k_mse<<<grid_for(d0.n()), 256, 0, n->stream>>>(w->y, t, src, o[0], o[1], o[2], d0, w->scale, 4, w->gy, w->loss);
  CHK(last_launch("k_mse"));
  CHK(net_backward(n, w));
  if (loss) {
    HIPCHK(hipMemcpyAsync(loss, w->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    HIPCHK(hipStreamSynchronize(n->stream));
  }
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_net_adam_step(mh3d_net_t n, float lr, float beta1, float beta2, float eps) {
  if (!n) return fail(MH3D_ERR_INVALID, "NULL network");
  n->step += 1;
  const float c1 = 1.f - powf(beta1, (float)n->step), c2 = 1.f - powf(beta2, (float)n->step);
  k_adam<<<grid_for(n->nparam), 256, 0, n->stream>>>(n->p, n->g, n->m, n->v, n->nparam, lr, beta1, beta2, eps, c1, c2);
  CHK(last_launch("k_adam"));
  CHK(net_pack(n));
  return MH3D_OK;
}

extern "C" mh3d_status mh3d_warm_start(mh3d_plan_t p, mh3d_net_t n, const float* d, float* rho_init) {
  CHK(check_plan(p));
  if (!n || !d || !rho_init) return fail(MH3D_ERR_INVALID, "NULL argument");
  const Geo& g = p->g;
  CHK(net_check_dims(n, g.nx, g.ny, g.nz));
  if (n->stream != p->stream) return fail(MH3D_ERR_INVALID, "network and plan must share a stream");
  if (n->in_ch != g.K) return fail(MH3D_ERR_INVALID, "network has %d input channels, plan %d harmonics", n->in_ch, g.K);
  NetWork* w;
  CHK(net_work(n, g.nx, g.ny, g.nz, &w));
  if (!w->xin) CHK(net_alloc((void**)&w->xin, sizeof(float) * (size_t)g.K * g.N));
  // per-harmonic back-projections c_k = b (H_k^T P^T d_k), the network's channels
  CHK(mh3d_backproject(p, d, w->xin));
  Dims src{ilog2(g.nx), ilog2(g.ny), ilog2(g.nz)};
  CHK(net_forward(n, w, w->xin, src, g.N, 0, 0, 0, true));
  k_scale_relu<<<grid_for(g.N), 256, 0, p->stream>>>(w->y, g.N, w->scale, rho_init);
  CHK(last_launch("k_scale_relu"));
  return MH3D_OK;
}

// ============================================================================ training data on the GPU
namespace {

// Object parameters drawn from Philox4x32-10: stream = object index, key = seed,
// counter (j, object, 0, 0) for the j-th block of four uniforms u = (w + 0.5)/2^32.
// Spheres (kind 0): radius U(2,5) mm, centre U(r, extent - r) per axis, concentration
// 10^U(-2,0).  Tubes (kind 1): radius U(1,2.5) mm, three Bezier points U(3, extent - 3),
// concentration 10^U(-2,0).
struct Obj {
  double c[9];     // sphere: centre[3]; tube: p0[3], p1[3], p2[3]
  double r, conc;
  int kind;
};

__device__ __forceinline__ double philox_u(uint64_t seed, uint32_t obj, uint32_t j, int w) {
  uint32_t c[4] = {j, obj, 0u, 0u};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  return ((double)c[w] + 0.5) / 4294967296.0;
}

__global__ void k_phantom_objects(uint64_t seed, int nsph, int ntube, double ex, double ey, double ez,
                                  Obj* __restrict__ objs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsph + ntube) return;
  Obj o;
  const double ext[3] = {ex, ey, ez};
  auto u = [&](int q) { return philox_u(seed, (uint32_t)i, (uint32_t)(q >> 2), q & 3); };
  if (i < nsph) {
    o.kind = 0;
    o.r = 2.0 + 3.0 * u(0);
    for (int a = 0; a < 3; ++a) o.c[a] = o.r + (ext[a] - 2.0 * o.r) * u(1 + a);
    o.conc = pow(10.0, -2.0 + 2.0 * u(4));
  } else {
    o.kind = 1;
    o.r = 1.0 + 1.5 * u(0);
    for (int q = 0; q < 9; ++q) o.c[q] = 3.0 + (ext[q % 3] - 6.0) * u(1 + q);
    o.conc = pow(10.0, -2.0 + 2.0 * u(10));
  }
  objs[i] = o;
}

// Tube membership by stamping: a voxel belongs to tube t when some sample of the
// curve (t = s/256, s = 0..256) lies within r of it, i.e. the nearest of the 257
// samples does.  One thread per (tube, sample) visits the voxels of the sample's
// r-box and sets bit t of the voxel's flag word.  tubes <= 32; tube t is object
// nsph + t.
__global__ void k_phantom_stamp(Geo g, double vox, const Obj* __restrict__ objs, int nsph, int ntube,
                                unsigned* __restrict__ flags) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ntube * 257) return;
  const int t = id / 257, s = id - t * 257;
  const Obj& o = objs[nsph + t];
  const double u = s / 256.0, a0 = (1 - u) * (1 - u), a1 = 2 * (1 - u) * u, a2 = u * u;
  const double cx = a0 * o.c[0] + a1 * o.c[3] + a2 * o.c[6];
  const double cy = a0 * o.c[1] + a1 * o.c[4] + a2 * o.c[7];
  const double cz = a0 * o.c[2] + a1 * o.c[5] + a2 * o.c[8];
  const int dims[3] = {g.nx, g.ny, g.nz};
  const double c[3] = {cx, cy, cz};
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int)ceil((c[a] - o.r) / vox) - 1;      // one voxel of slack each side: the
    hi[a] = (int)floor((c[a] + o.r) / vox) + 1;     // distance test below decides
    lo[a] = lo[a] < 0 ? 0 : lo[a];
    hi[a] = hi[a] > dims[a] - 1 ? dims[a] - 1 : hi[a];
  }
  for (int x = lo[0]; x <= hi[0]; ++x)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int z = lo[2]; z <= hi[2]; ++z) {
        const double px = x * vox, py = y * vox, pz = z * vox;
        const double d2 = (px - cx) * (px - cx) + (py - cy) * (py - cy) + (pz - cz) * (pz - cz);
        if (d2 <= o.r * o.r) atomicOr(&flags[((long long)x * g.ny + y) * g.nz + z], 1u << t);
      }
}

// Voxel-centre inclusion (centres at i * voxel); overlapping objects add, in object
// order, in FP64.  Tube distance: nearest of 257 samples of the curve (from the
// stamped flags when given, else by direct search).
__global__ void k_phantom_raster(Geo g, double vox, const Obj* __restrict__ objs, int nobj,
                                 const unsigned* __restrict__ flags, int nsph, float* __restrict__ rho) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < g.N; i += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(i % g.nz);
    const int y = (int)((i / g.nz) % g.ny);
    const int x = (int)(i / ((long long)g.ny * g.nz));
    const double px = x * vox, py = y * vox, pz = z * vox;
    double acc = 0.0;
    for (int q = 0; q < nobj; ++q) {
      const Obj& o = objs[q];
      if (o.kind == 0) {
        const double dx = px - o.c[0], dy = py - o.c[1], dz = pz - o.c[2];
        if (dx * dx + dy * dy + dz * dz <= o.r * o.r) acc += o.conc;
      } else if (flags) {
        if ((flags[i] >> (q - nsph)) & 1u) acc += o.conc;
      } else {
        // bounding box of the control polygon (contains the curve) grown by r
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = fmin(fmin(o.c[a], o.c[3 + a]), o.c[6 + a]) - o.r;
          hi[a] = fmax(fmax(o.c[a], o.c[3 + a]), o.c[6 + a]) + o.r;
        }
        if (px < lo[0] || px > hi[0] || py < lo[1] || py > hi[1] || pz < lo[2] || pz > hi[2]) continue;
        double best = 1e300;
        for (int s = 0; s <= 256; ++s) {
          const double t = s / 256.0, a0 = (1 - t) * (1 - t), a1 = 2 * (1 - t) * t, a2 = t * t;
          const double cx = a0 * o.c[0] + a1 * o.c[3] + a2 * o.c[6];
          const double cy = a0 * o.c[1] + a1 * o.c[4] + a2 * o.c[7];
          const double cz = a0 * o.c[2] + a1 * o.c[5] + a2 * o.c[8];
          const double d2 = (px - cx) * (px - cx) + (py - cy) * (py - cy) + (pz - cz) * (pz - cz);
          best = fmin(best, d2);
        }
        if (best <= o.r * o.r) acc += o.conc;
      }
    }
    rho[i] = (float)acc;
  }
}

// Per-harmonic mean square of the portraits (FP64, one block per harmonic).
__global__ void k_port_meansq(const float* __restrict__ d, long long M, double* __restrict__ ms) {
  __shared__ double part[256];
  const int k = blockIdx.x;
  double s = 0.0;
  for (long long i = threadIdx.x; i < M; i += blockDim.x) {
    const double v = d[(long long)k * M + i];
    s += v * v;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < (int)blockDim.x; ++q) t += part[q];
    ms[k] = t / (double)M;
  }
}

// d_k += sigma_k xi, sigma_k = rms_k 10^(-(snr2 - decay (k_idx... )) / 20), xi standard
// normal by Box-Muller from Philox stream (seed, 1): counter (i/2, 1, 0, 0).
__global__ void k_add_noise(float* __restrict__ d, long long M, int K, const double* __restrict__ ms,
                            const int* __restrict__ harm, double snr2, double decay, uint64_t seed) {
  const long long n = (long long)K * M;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(i / M);
    uint32_t c[4] = {(uint32_t)(i >> 1), 1u, (uint32_t)(i >> 33), 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    const double u1 = ((double)c[(i & 1) * 2] + 0.5) / 4294967296.0;
    const double u2 = ((double)c[(i & 1) * 2 + 1] + 0.5) / 4294967296.0;
    const double xi = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
    const double snr = snr2 - decay * (harm[k] - 2);
    const double sigma = sqrt(ms[k]) * pow(10.0, -snr / 20.0);
    d[i] = (float)(d[i] + sigma * xi);
  }
}

}  // namespace

extern "C" mh3d_status mh3d_phantom(mh3d_plan_t p, uint64_t seed, int32_t n_spheres, int32_t n_tubes, float* rho) {
  CHK(check_plan(p));
  if (!rho || n_spheres < 0 || n_tubes < 0 || n_spheres + n_tubes > 4096)
    return fail(MH3D_ERR_INVALID, "bad phantom arguments");
  const Geo& g = p->g;
  const int nobj = n_spheres + n_tubes;
  Obj* objs = nullptr;
  HIPCHK(hipMalloc(&objs, sizeof(Obj) * (nobj > 0 ? nobj : 1)));
  unsigned* flags = nullptr;
  if (n_tubes > 0 && n_tubes <= 32) {
    if (hipMalloc(&flags, sizeof(unsigned) * (size_t)g.N) != hipSuccess) {
      (void)hipFree(objs);
      return fail(MH3D_ERR_OOM, "phantom flags");
    }
    (void)hipMemsetAsync(flags, 0, sizeof(unsigned) * (size_t)g.N, p->stream);
  }
  const double v = p->desc.voxel_mm;
  if (nobj)
    k_phantom_objects<<<(nobj + 63) / 64, 64, 0, p->stream>>>(seed, n_spheres, n_tubes, (g.nx - 1) * v,
                                                             (g.ny - 1) * v, (g.nz - 1) * v, objs);
  if (flags) k_phantom_stamp<<<(n_tubes * 257 + 63) / 64, 64, 0, p->stream>>>(g, v, objs, n_spheres, n_tubes, flags);
  k_phantom_raster<<<grid_for(g.N), 256, 0, p->stream>>>(g, v, objs, nobj, flags, n_spheres, rho);
  mh3d_status s = last_launch("k_phantom_raster");
  if (hipStreamSynchronize(p->stream) != hipSuccess && s == MH3D_OK) s = fail(MH3D_ERR_HIP, "phantom kernel failed");
  (void)hipFree(objs);
  if (flags) (void)hipFree(flags);
  return s;
}

extern "C" mh3d_status mh3d_noisy_data(mh3d_plan_t p, const float* rho, uint64_t seed, double snr2_db,
                                       double decay_db, float* d) {
  CHK(check_plan(p));
  if (!rho || !d) return fail(MH3D_ERR_INVALID, "NULL argument");
  const Geo& g = p->g;
  CHK(mh3d_forward(p, rho, d));
  double* ms = nullptr;
  int* harm = nullptr;
  HIPCHK(hipMalloc(&ms, sizeof(double) * g.K));
  HIPCHK(hipMalloc(&harm, sizeof(int) * g.K));
  HIPCHK(hipMemcpyAsync(harm, p->harm.data(), sizeof(int) * g.K, hipMemcpyHostToDevice, p->stream));
  k_port_meansq<<<g.K, 256, 0, p->stream>>>(d, g.Mf, ms);
  mh3d_status s = last_launch("k_port_meansq");
  if (s == MH3D_OK) {
    k_add_noise<<<grid_for((long long)g.K * g.Mf), 256, 0, p->stream>>>(d, g.Mf, g.K, ms, harm, snr2_db, decay_db, seed);
    s = last_launch("k_add_noise");
  }
  if (hipStreamSynchronize(p->stream) != hipSuccess && s == MH3D_OK) s = fail(MH3D_ERR_HIP, "noise kernel failed");
  (void)hipFree(ms);
  (void)hipFree(harm);
  return s;
}
