// Host side of the warm-start network: layer plan, workspace layout and the
// launch sequences of inference, loss gradient and Adam.  Included inside the
// library's internal namespace of rism3d.hip (uses fail / HIP_TRY / TIMED).
//
// Architecture (levels L, channels C_l = base * 2^l, 3x3x3 convolutions with
// zero padding, leaky activations, 2x2x2 average pooling, nearest upsampling):
//   encoder l:  a_l = act(conv(in_l)), e_l = act(conv(a_l)), in_0 = input,
//               in_{l+1} = pool(e_l);
//   decoder l = L-2 .. 0:  da_l = act(conv([up(d_{l+1}), e_l])), d_l = act(conv(da_l)),
//               d_{L-1} = e_{L-1};
//   output = conv(d_0).
// Parameters (FP32, flat): per convolution in the order enc0a, enc0b, ...,
// enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b, out: W[C_out][27][C_in]
// (tap k = (dz * 3 + dy) * 3 + dx for offsets (dz-1, dy-1, dx-1)) then b[C_out].

struct NetLayer {
  int cin, cout;          // real channel counts
  int cin_pad, cout_pad;  // packed: cin to a multiple of 8, cout to a multiple of 16
  int level;
  size_t w_off, b_off;    // offsets in the parameter vector (floats)
  size_t wp, wf;          // workspace offsets of the packed and flipped BF16 weights
};

constexpr int kNetMaxLevels = 6;

struct NetPlan {
  rism3d_unet_config cfg;
  int nz[kNetMaxLevels], ny[kNetMaxLevels], nx[kNetMaxLevels];
  size_t nvox[kNetMaxLevels];
  std::vector<NetLayer> layers;
  size_t n_params = 0;
  size_t x0 = 0, a[kNetMaxLevels] = {}, e[kNetMaxLevels] = {}, p[kNetMaxLevels] = {},
         da[kNetMaxLevels] = {}, db[kNetMaxLevels] = {};
  size_t out = 0, ge[kNetMaxLevels] = {}, gd[kNetMaxLevels] = {}, gtmp = 0, gdx = 0, dyp = 0,
         partials = 0, loss = 0, slabs = 0;
  size_t total_infer = 0, total_train = 0;
  int c(int l) const { return cfg.base << l; }
};

constexpr int kMsePartials = 1024;

// Workgroups per tap of the weight gradient over N voxels (chunks of
// kWgradChunk voxels, about 96 workgroups x 27 taps at full size), and the
// voxel chunks each one takes.
size_t wgrad_per(size_t N) {
  const size_t chunks_total = (N + net::kWgradChunk - 1) / net::kWgradChunk;
  const size_t wg_target = 96;
  return std::max<size_t>(1, (chunks_total + wg_target - 1) / wg_target);
}
size_t wgrad_blocks(size_t N) {
  const size_t chunks_total = (N + net::kWgradChunk - 1) / net::kWgradChunk;
  return (chunks_total + wgrad_per(N) - 1) / wgrad_per(N);
}
size_t bias_blocks(size_t N, int cout_pad) {
  const size_t per_block = (size_t)(net::kConvThreads / cout_pad);
  return std::min<size_t>(1024, (N + per_block - 1) / per_block);
}

rism3d_status net_plan(const rism3d_unet_config* cfg, int nx, int ny, int nz, NetPlan* P) {
  if (!cfg) return fail(RISM3D_E_ARG, "null network configuration");
  const int L = cfg->levels;
  if (L < 1 || L > kNetMaxLevels) return fail(RISM3D_E_ARG, "levels must be in 1..%d", kNetMaxLevels);
  // (the weight-gradient kernel holds at most 64 16x16 tiles per workgroup:
  // 128 x 128 and 192 x 64 channel pairs at base 16, 4 levels)
  if (cfg->base < 16 || cfg->base % 16 || (cfg->base << (L - 1)) > 128)
    return fail(RISM3D_E_ARG, "base channels must be a multiple of 16 with base * 2^(levels-1) <= 128");
  if (cfg->in_channels < 1 || cfg->in_channels > 64 || cfg->out_channels < 1 ||
      cfg->out_channels > 64)
    return fail(RISM3D_E_ARG, "in/out channels must be in 1..64");
  if (!(cfg->slope >= 0.0f && cfg->slope < 1.0f)) return fail(RISM3D_E_ARG, "slope must be in [0, 1)");
  const int m = 1 << (L - 1);
  if (nx < m || ny < m || nz < m || nx % m || ny % m || nz % m)
    return fail(RISM3D_E_ARG, "grid %dx%dx%d: every axis must be a positive multiple of %d", nx, ny,
                nz, m);
  if ((size_t)nx * ny * nz > ((size_t)1 << 30))
    return fail(RISM3D_E_ARG, "grid too large for the network");
  P->cfg = *cfg;
  for (int l = 0; l < L; ++l) {
    P->nx[l] = nx >> l;
    P->ny[l] = ny >> l;
    P->nz[l] = nz >> l;
    P->nvox[l] = (size_t)P->nx[l] * P->ny[l] * P->nz[l];
  }
  P->layers.clear();
  auto add = [&](int cin, int cout, int level) {
    NetLayer ly;
    ly.cin = cin;
    ly.cout = cout;
    ly.cin_pad = (cin + 7) & ~7;
    ly.cout_pad = (cout + 15) & ~15;
    ly.level = level;
    ly.w_off = P->n_params;
    P->n_params += (size_t)cout * 27 * cin;
    ly.b_off = P->n_params;
    P->n_params += cout;
    P->layers.push_back(ly);
  };
  P->n_params = 0;
  for (int l = 0; l < L; ++l) {
    add(l == 0 ? cfg->in_channels : P->c(l - 1), P->c(l), l);
    add(P->c(l), P->c(l), l);
  }
  for (int l = L - 2; l >= 0; --l) {
    add(P->c(l + 1) + P->c(l), P->c(l), l);
    add(P->c(l), P->c(l), l);
  }
  add(P->c(0), cfg->out_channels, 0);
  for (const NetLayer& ly : P->layers)
    if ((ly.cout_pad / 16) * ((ly.cin_pad + 15) / 16) > 4 * net::kWgradMaxTiles)
      return fail(RISM3D_E_ARG, "layer %d x %d channels exceeds the weight-gradient tile budget",
                  ly.cin, ly.cout);

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  for (NetLayer& ly : P->layers) {
    ly.wp = take((size_t)ly.cout_pad * 27 * ly.cin_pad * 2);
    ly.wf = take((size_t)((ly.cin + 15) & ~15) * 27 * ly.cout_pad * 2);
  }
  P->x0 = take(P->nvox[0] * P->layers[0].cin_pad * 2);
  for (int l = 0; l < L; ++l) {
    if (l > 0) P->p[l] = take(P->nvox[l] * P->c(l - 1) * 2);
    P->a[l] = take(P->nvox[l] * P->c(l) * 2);
    P->e[l] = take(P->nvox[l] * P->c(l) * 2);
  }
  for (int l = L - 2; l >= 0; --l) {
    P->da[l] = take(P->nvox[l] * P->c(l) * 2);
    P->db[l] = take(P->nvox[l] * P->c(l) * 2);
  }
  P->total_infer = off;
  P->out = take(P->nvox[0] * cfg->out_channels * 4);
  size_t max_c = 0, max_cin = 0, max_cout_pad = 0;
  for (const NetLayer& ly : P->layers) {
    max_c = std::max(max_c, P->nvox[ly.level] * (size_t)ly.cout);
    max_cin = std::max(max_cin, P->nvox[ly.level] * (size_t)((ly.cin + 15) & ~15));
    max_cout_pad = std::max(max_cout_pad, P->nvox[ly.level] * (size_t)ly.cout_pad);
  }
  for (int l = 0; l < L; ++l) {
    P->ge[l] = take(P->nvox[l] * P->c(l) * 4);
    if (l < L - 1) P->gd[l] = take(P->nvox[l] * P->c(l) * 4);
  }
  P->gtmp = take(max_c * 4);
  P->gdx = take(max_cin * 4);
  P->dyp = take(max_cout_pad * 2);
  P->partials = take(kMsePartials * sizeof(double));
  P->loss = take(sizeof(double));
  size_t slab_floats = 0;   // partial slabs of the largest weight (or bias) gradient
  for (const NetLayer& ly : P->layers) {
    const size_t w = wgrad_blocks(P->nvox[ly.level]) * (size_t)ly.cout * 27 * ly.cin;
    const size_t b = bias_blocks(P->nvox[ly.level], ly.cout_pad) * (size_t)ly.cout;
    slab_floats = std::max(slab_floats, std::max(w, b));
  }
  P->slabs = take(slab_floats * sizeof(float));
  P->total_train = off;
  return RISM3D_OK;
}

template <typename T>
T* wsp(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

unsigned net_blocks(size_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

void net_pack(const NetPlan& P, const float* params, void* ws, bool flipped, hipStream_t s) {
  for (const NetLayer& ly : P.layers) {
    const int cin16 = (ly.cin + 15) & ~15;
    const size_t n = (size_t)ly.cout_pad * 27 * ly.cin_pad +
                     (flipped ? (size_t)cin16 * 27 * ly.cout_pad : 0);
    hipLaunchKernelGGL(net::k_pack_weights, dim3(net_blocks(n, 256)), dim3(256), 0, s,
                       params + ly.w_off, ly.cout, ly.cin, ly.cout_pad, ly.cin_pad, cin16,
                       wsp<uint16_t>(ws, ly.wp), flipped ? wsp<uint16_t>(ws, ly.wf) : nullptr);
  }
}

// One convolution (channel counts are multiples of 8): the halo-tiled
// kernel, staging CGC <= 4 channel groups (at most 64 KB of LDS) at a time,
// CGC the largest of 4, 3, 2, 1 that divides the group count.  Tiles of
// 16 x 8 x 4 voxels, or 16 x 2 x 4 where those would give fewer than 512
// workgroups (the coarse levels).
template <int EPI, int CGC, int TY>
void net_conv_tiles(const net::ConvArgs& a, unsigned tiles, hipStream_t s) {
  hipLaunchKernelGGL((net::k_conv3<EPI, CGC, TY>), dim3(tiles, a.cout_pad / 16),
                     dim3(net::kConvThreads), 0, s, a);
}

template <int EPI, int CGC>
void net_conv_chunks(const net::ConvArgs& a, hipStream_t s) {
  auto tiles = [&](int ty) {
    return (unsigned)((a.nx + net::kTileX - 1) / net::kTileX) * (unsigned)((a.ny + ty - 1) / ty) *
           (unsigned)((a.nz + net::kTileZ - 1) / net::kTileZ);
  };
  if (tiles(8) * (unsigned)(a.cout_pad / 16) >= 512) net_conv_tiles<EPI, CGC, 8>(a, tiles(8), s);
  else net_conv_tiles<EPI, CGC, 2>(a, tiles(2), s);
}

template <int EPI>
void net_conv(const net::ConvArgs& a, hipStream_t s) {
  const int cg = (a.in.ca + a.in.cb) / 8;
  if (cg % 4 == 0) net_conv_chunks<EPI, 4>(a, s);
  else if (cg % 3 == 0) net_conv_chunks<EPI, 3>(a, s);
  else if (cg % 2 == 0) net_conv_chunks<EPI, 2>(a, s);
  else net_conv_chunks<EPI, 1>(a, s);
}

net::ConvArgs conv_args(const NetPlan& P, const NetLayer& ly, void* ws, net::ConvIn in,
                        const float* params) {
  net::ConvArgs a;
  a.in = in;
  a.w = wsp<uint16_t>(ws, ly.wp);
  a.bias = params + ly.b_off;
  a.yb = nullptr;
  a.yf = nullptr;
  a.cout = ly.cout;
  a.cout_pad = ly.cout_pad;
  a.nz = P.nz[ly.level];
  a.ny = P.ny[ly.level];
  a.nx = P.nx[ly.level];
  a.slope = P.cfg.slope;
  return a;
}

// Inputs of every convolution in parameter order (needed again by the
// weight gradients).
std::vector<net::ConvIn> net_inputs(const NetPlan& P, void* ws) {
  const int L = P.cfg.levels;
  std::vector<net::ConvIn> in;
  for (int l = 0; l < L; ++l) {
    if (l == 0) in.push_back({wsp<uint16_t>(ws, P.x0), nullptr, P.layers[0].cin_pad, 0, 0});
    else in.push_back({wsp<uint16_t>(ws, P.p[l]), nullptr, P.c(l - 1), 0, 0});
    in.push_back({wsp<uint16_t>(ws, P.a[l]), nullptr, P.c(l), 0, 0});
  }
  for (int l = L - 2; l >= 0; --l) {
    const size_t dprev = (l == L - 2) ? P.e[L - 1] : P.db[l + 1];
    in.push_back({wsp<uint16_t>(ws, dprev), wsp<uint16_t>(ws, P.e[l]), P.c(l + 1), P.c(l), 1});
    in.push_back({wsp<uint16_t>(ws, P.da[l]), nullptr, P.c(l), 0, 0});
  }
  in.push_back({wsp<uint16_t>(ws, L >= 2 ? P.db[0] : P.e[0]), nullptr, P.c(0), 0, 0});
  return in;
}

// Output tensor (BF16 activation) of every hidden convolution.
std::vector<size_t> net_outputs(const NetPlan& P) {
  const int L = P.cfg.levels;
  std::vector<size_t> out;
  for (int l = 0; l < L; ++l) {
    out.push_back(P.a[l]);
    out.push_back(P.e[l]);
  }
  for (int l = L - 2; l >= 0; --l) {
    out.push_back(P.da[l]);
    out.push_back(P.db[l]);
  }
  return out;
}

// Forward pass: input FP32 site-major [in_channels][N0] -> out FP32
// site-major [out_channels][N0].  Weights must be packed (net_pack).
void net_forward(const NetPlan& P, const float* params, const float* input, float* out, void* ws,
                 hipStream_t s) {
  const int L = P.cfg.levels;
  const NetLayer& l0 = P.layers[0];
  hipLaunchKernelGGL(net::k_to_channels_last, dim3(net_blocks(P.nvox[0] * l0.cin_pad, 256)),
                     dim3(256), 0, s, input, P.cfg.in_channels, l0.cin_pad, P.nvox[0],
                     wsp<uint16_t>(ws, P.x0));
  const std::vector<net::ConvIn> in = net_inputs(P, ws);
  const std::vector<size_t> outs = net_outputs(P);
  for (size_t j = 0; j + 1 < P.layers.size(); ++j) {
    const NetLayer& ly = P.layers[j];
    if (j >= 2 && j < (size_t)2 * L && j % 2 == 0) {   // encoder level l = j / 2 >= 1: pool e_{l-1}
      const int l = (int)j / 2;
      hipLaunchKernelGGL(net::k_pool2, dim3(net_blocks(P.nvox[l] * (P.c(l - 1) / 8), 256)),
                         dim3(256), 0, s, wsp<uint16_t>(ws, P.e[l - 1]), wsp<uint16_t>(ws, P.p[l]),
                         P.nz[l - 1], P.ny[l - 1], P.nx[l - 1], P.c(l - 1));
    }
    net::ConvArgs a = conv_args(P, ly, ws, in[j], params);
    a.yb = wsp<uint16_t>(ws, outs[j]);
    net_conv<net::EPI_BF16_LEAKY>(a, s);
  }
  const NetLayer& lo = P.layers.back();
  net::ConvArgs a = conv_args(P, lo, ws, in.back(), params);
  a.yf = out;
  net_conv<net::EPI_F32_SITE>(a, s);
}

// dX of one convolution (transposed convolution of dy_pre with the flipped
// weights) into FP32 channels last [N][cin].
void net_conv_dx(const NetPlan& P, const NetLayer& ly, void* ws, const uint16_t* dyp, float* dx,
                 hipStream_t s) {
  net::ConvArgs a;
  a.in = {dyp, nullptr, ly.cout_pad, 0, 0};
  a.w = wsp<uint16_t>(ws, ly.wf);
  a.bias = nullptr;
  a.yb = nullptr;
  a.yf = dx;
  a.cout = ly.cin;
  a.cout_pad = (ly.cin + 15) & ~15;
  a.nz = P.nz[ly.level];
  a.ny = P.ny[ly.level];
  a.nx = P.nx[ly.level];
  a.slope = 0.0f;
  net_conv<net::EPI_F32_CL>(a, s);
}

void net_conv_dw(const NetPlan& P, const NetLayer& ly, const net::ConvIn& in, void* ws,
                 const uint16_t* dyp, float* grad, hipStream_t s) {
  const size_t N = P.nvox[ly.level];
  const size_t per = wgrad_per(N);
  const size_t nbx = wgrad_blocks(N);
  float* slabs = wsp<float>(ws, P.slabs);
  net::WgradArgs w;
  w.in = in;
  w.dy = dyp;
  w.dw = slabs;
  w.cin_real = ly.cin;
  w.cout = ly.cout;
  w.cout_pad = ly.cout_pad;
  w.nz = P.nz[ly.level];
  w.ny = P.ny[ly.level];
  w.nx = P.nx[ly.level];
  w.chunks = (int)per;
  const int cit = (ly.cin_pad + 15) / 16;
  const int R = net::wgrad_group((ly.cout_pad / 16) * cit);
  const size_t lds = ((size_t)ly.cout_pad + (size_t)cit * 16) * net::wgrad_pitch(R) * 2;
  const dim3 grid((unsigned)nbx, 27), block(net::kConvThreads);
  if (R == 4) hipLaunchKernelGGL(net::k_conv3_wgrad<4>, grid, block, lds, s, w);
  else hipLaunchKernelGGL(net::k_conv3_wgrad<1>, grid, block, lds, s, w);
  const size_t nw = (size_t)ly.cout * 27 * ly.cin;
  hipLaunchKernelGGL(net::k_sum_slabs, dim3(net_blocks(nw, 256)), dim3(256), 0, s, slabs,
                     (int)nbx, nw, grad + ly.w_off);
  const unsigned nb = (unsigned)bias_blocks(N, ly.cout_pad);
  hipLaunchKernelGGL(net::k_bias_grad, dim3(nb), dim3(net::kConvThreads), 0, s, dyp, (int)N,
                     ly.cout, ly.cout_pad, slabs);
  hipLaunchKernelGGL(net::k_sum_slabs, dim3(net_blocks(ly.cout, 256)), dim3(256), 0, s, slabs,
                     (int)nb, (size_t)ly.cout, grad + ly.b_off);
}

void net_leaky_bwd(const NetPlan& P, size_t y_off, const float* g, int level, int C, void* ws,
                   hipStream_t s) {
  const size_t n = P.nvox[level] * C;
  hipLaunchKernelGGL(net::k_leaky_bwd, dim3(net_blocks(n, 256)), dim3(256), 0, s,
                     wsp<uint16_t>(ws, y_off), g, wsp<uint16_t>(ws, P.dyp), n, P.cfg.slope);
}

// Loss (mean squared error against target, FP32 site-major) and its
// gradient with respect to every parameter (grad, FP32, overwritten).
void net_gradient(const NetPlan& P, const float* params, const float* input, const float* target,
                  float* grad, void* ws, hipStream_t s) {
  const int L = P.cfg.levels;
  float* out = wsp<float>(ws, P.out);
  net_forward(P, params, input, out, ws, s);
  hipLaunchKernelGGL(net::k_fill_f32, dim3(net_blocks(P.n_params, 256)), dim3(256), 0, s, grad,
                     P.n_params, 0.0f);
  const NetLayer& lo = P.layers.back();
  hipLaunchKernelGGL(net::k_mse, dim3(kMsePartials), dim3(256), 0, s, out, target, lo.cout,
                     lo.cout_pad, P.nvox[0], wsp<uint16_t>(ws, P.dyp), wsp<double>(ws, P.partials));
  hipLaunchKernelGGL(net::k_sum_partials, dim3(1), dim3(64), 0, s, wsp<double>(ws, P.partials),
                     kMsePartials, 1.0 / ((double)lo.cout * (double)P.nvox[0]),
                     wsp<double>(ws, P.loss));
  const std::vector<net::ConvIn> in = net_inputs(P, ws);
  const std::vector<size_t> outs = net_outputs(P);
  const uint16_t* dyp = wsp<uint16_t>(ws, P.dyp);
  float* gtmp = wsp<float>(ws, P.gtmp);
  float* gdx = wsp<float>(ws, P.gdx);
  const size_t jo = P.layers.size() - 1;
  net_conv_dw(P, lo, in[jo], ws, dyp, grad, s);
  // gradient at d_0 (or e_0 when there is a single level)
  float* g_top = wsp<float>(ws, L >= 2 ? P.gd[0] : P.ge[0]);
  net_conv_dx(P, lo, ws, dyp, g_top, s);
  for (int l = 0; l <= L - 2; ++l) {
    const size_t jb = jo - 1 - 2 * (size_t)l, ja = jb - 1;
    const NetLayer& lb = P.layers[jb];
    const NetLayer& la = P.layers[ja];
    net_leaky_bwd(P, outs[jb], wsp<float>(ws, P.gd[l]), l, P.c(l), ws, s);
    net_conv_dw(P, lb, in[jb], ws, dyp, grad, s);
    net_conv_dx(P, lb, ws, dyp, gtmp, s);
    net_leaky_bwd(P, outs[ja], gtmp, l, P.c(l), ws, s);
    net_conv_dw(P, la, in[ja], ws, dyp, grad, s);
    net_conv_dx(P, la, ws, dyp, gdx, s);
    const int cin = la.cin, ca = P.c(l + 1);
    hipLaunchKernelGGL(net::k_take_skip, dim3(net_blocks(P.nvox[l] * (cin - ca), 256)), dim3(256),
                       0, s, gdx, cin, ca, wsp<float>(ws, P.ge[l]), P.nvox[l]);
    float* gup = wsp<float>(ws, (l + 1 == L - 1) ? P.ge[L - 1] : P.gd[l + 1]);
    hipLaunchKernelGGL(net::k_up2_bwd, dim3(net_blocks(P.nvox[l + 1] * ca, 256)), dim3(256), 0, s,
                       gdx, cin, ca, gup, P.nz[l], P.ny[l], P.nx[l]);
  }
  for (int l = L - 1; l >= 0; --l) {
    const NetLayer& lb = P.layers[2 * l + 1];
    const NetLayer& la = P.layers[2 * l];
    net_leaky_bwd(P, outs[2 * l + 1], wsp<float>(ws, P.ge[l]), l, P.c(l), ws, s);
    net_conv_dw(P, lb, in[2 * l + 1], ws, dyp, grad, s);
    net_conv_dx(P, lb, ws, dyp, gtmp, s);
    net_leaky_bwd(P, outs[2 * l], gtmp, l, P.c(l), ws, s);
    net_conv_dw(P, la, in[2 * l], ws, dyp, grad, s);
    if (l > 0) {
      net_conv_dx(P, la, ws, dyp, gdx, s);
      const size_t n = P.nvox[l - 1] * P.c(l - 1);
      hipLaunchKernelGGL(net::k_pool2_bwd_add, dim3(net_blocks(n, 256)), dim3(256), 0, s, gdx,
                         wsp<float>(ws, P.ge[l - 1]), P.nz[l - 1], P.ny[l - 1], P.nx[l - 1],
                         P.c(l - 1));
    }
  }
}
