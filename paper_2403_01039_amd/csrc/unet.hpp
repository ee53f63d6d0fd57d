// Warm-start network kernels for gfx950.
//
// The network (a 3D convolutional encoder-decoder, see unet_host.hpp) maps the
// solute potential of each solvent site to an initial short-range direct
// correlation; the paper itself starts every solve at t = f.  Activations are
// BF16, channels last ([voxel][channel], channel count a multiple of 8), so 8
// channels of one voxel are one 16-byte load.  The 3x3x3 convolutions are
// implicit GEMMs on the matrix cores:
//   v_mfma_f32_16x16x32_bf16:  D[16x16] += A[16x32] B[32x16], FP32 accumulate,
//   A = packed weights (rows = output channels), B = input voxels (columns),
//   K = (tap, input channel) with 8 consecutive channels per lane.
// Lane l supplies row/column (l & 15) and the K slice 8 (l >> 4) .. +7 of its
// operand; it receives D rows 4 (l >> 4) .. +3 of column (l & 15), i.e. four
// consecutive output channels of one voxel (one 8-byte BF16 store).
// Weight gradients use the same instruction on LDS-transposed tiles.
#pragma once

#include "common.hpp"

namespace rism {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kConvThreads = 256;   // 4 waves
constexpr int kWgradChunk = 64;     // voxels per LDS tile of the weight gradient
constexpr int kWgradMaxTiles = 16;  // 16x16 output tiles per wave

// FP32 -> BF16 with round-to-nearest-even (NaN stays NaN); BF16 -> FP32 exact.
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {   // 16-byte aligned
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() {
  const u32x4 z = {0u, 0u, 0u, 0u};
  return __builtin_bit_cast(bf16x8, z);
}

// Offsets of tap k = (dz * 3 + dy) * 3 + dx are (dz - 1, dy - 1, dx - 1).
__device__ __forceinline__ void tap_offset(int tap, int& dz, int& dy, int& dx) {
  dz = tap / 9 - 1;
  dy = (tap / 3) % 3 - 1;
  dx = tap % 3 - 1;
}

// Input of a convolution: channels [0, ca) from tensor a (on the output grid,
// or on the half grid and read through nearest-neighbour upsampling when
// up_a), channels [ca, ca + cb) from tensor b (the skip branch).
struct ConvIn {
  const uint16_t* a;
  const uint16_t* b;
  int ca, cb, up_a;
};

// 8 channels (group cg) of voxel (z, y, x) of the virtual input; zero outside.
__device__ __forceinline__ bf16x8 load_in(const ConvIn& in, int cg, int z, int y, int x, int nz,
                                          int ny, int nx) {
  if ((unsigned)z >= (unsigned)nz || (unsigned)y >= (unsigned)ny || (unsigned)x >= (unsigned)nx)
    return zero8();
  const int c = cg * 8;
  if (c < in.ca) {
    const size_t v = in.up_a ? ((size_t)(z >> 1) * (ny >> 1) + (y >> 1)) * (nx >> 1) + (x >> 1)
                             : ((size_t)z * ny + y) * nx + x;
    return ld8(in.a + v * in.ca + c);
  }
  return ld8(in.b + (((size_t)z * ny + y) * nx + x) * in.cb + (c - in.ca));
}

enum ConvEpilogue {
  EPI_BF16_LEAKY = 0,   // + bias, leaky, BF16 channels last [N][cout_pad]
  EPI_F32_SITE = 1,     // + bias, FP32 site-major [cout][N] (channels < cout)
  EPI_F32_CL = 2,       // raw FP32 channels last [N][cout_pad]
};

struct ConvArgs {
  ConvIn in;
  const uint16_t* w;    // packed [cout_pad][27][cin], cin = ca + cb
  const float* bias;    // [cout] (EPI 0, 1)
  uint16_t* yb;         // EPI_BF16_LEAKY output
  float* yf;            // EPI_F32_SITE / EPI_F32_CL output
  int cout, cout_pad;
  int nz, ny, nx;
  float slope;
};

// Epilogue of one accumulator tile: output channels c0 .. c0 + 3 of voxel v.
template <int EPI>
__device__ __forceinline__ void conv_store(const ConvArgs& p, int N, size_t v, int c0,
                                           const f32x4& r) {
  if (EPI == EPI_BF16_LEAKY) {
    uint16_t h[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float val = r[e] + (c0 + e < p.cout ? p.bias[c0 + e] : 0.0f);
      val = val > 0.0f ? val : p.slope * val;
      h[e] = f2bf(val);
    }
    const u32x2 pk = {(uint32_t)h[0] | ((uint32_t)h[1] << 16),
                      (uint32_t)h[2] | ((uint32_t)h[3] << 16)};
    *reinterpret_cast<u32x2*>(p.yb + v * p.cout_pad + c0) = pk;
  } else if (EPI == EPI_F32_SITE) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (c0 + e < p.cout) p.yf[(size_t)(c0 + e) * N + v] = r[e] + p.bias[c0 + e];
  } else {
    *reinterpret_cast<f32x4*>(p.yf + v * p.cout_pad + c0) = r;
  }
}

// Convolutions with 8 * CG input channels on a halo-tiled grid: a workgroup
// computes 16 output channels (tile blockIdx.y) of a 16 x TY x 4 voxel tile
// (TY = 8; 2 on small grids, for more workgroups).  It stages the tile's input
// with a one-voxel halo (18 x (TY + 2) x 6 voxels) in LDS, CGC channel groups at a
// time (CG / CGC chunks), and every tap's operand is read from there instead
// of from the cache hierarchy.  LDS layout [hz][hy][cg][hx] (16-byte units):
// the 16 voxels of one operand are consecutive units, conflict-free.  Wave w
// owns the z-slice z0 + w: its TY rows y0 .. y0 + TY - 1 of 16 voxels are its
// TY accumulator tiles.  Within a chunk the K steps take (tap, channel group)
// pairs in tap-major order, four per matrix instruction: lane group g
// supplies pair q0 + g (its 8 channels), the weights are the A operand (rows
// = output channels), the voxels the B operand (columns).
constexpr int kTileX = 16, kTileZ = 4;
constexpr int kHaloX = kTileX + 2, kHaloZ = kTileZ + 2;

template <int EPI, int CGC, int TY>
__global__ __launch_bounds__(kConvThreads) void k_conv3(ConvArgs p) {
  constexpr int kTileY = TY, kHaloY = TY + 2;
  __shared__ __align__(16) u32x4 halo[kHaloZ * kHaloY * CGC * kHaloX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int N = p.nz * p.ny * p.nx;
  const int CG = (p.in.ca + p.in.cb) >> 3;   // a multiple of CGC
  const int tiles_x = (p.nx + kTileX - 1) / kTileX, tiles_y = (p.ny + kTileY - 1) / kTileY;
  int b = (int)blockIdx.x;
  const int x0 = (b % tiles_x) * kTileX;
  b /= tiles_x;
  const int y0 = (b % tiles_y) * kTileY;
  const int z0 = (b / tiles_y) * kTileZ;
  const int cbase = (int)blockIdx.y * 16;
  f32x4 acc[kTileY];
#pragma unroll
  for (int t = 0; t < kTileY; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int nq = 27 * CGC;
  const size_t wrow = (size_t)27 * CG * 8;
  for (int c0 = 0; c0 < CG; c0 += CGC) {
    if (c0 > 0) __syncthreads();   // the previous chunk's operands are read
    // stage: item (h, cg), channel group fastest (consecutive 16-byte reads)
    for (int it = threadIdx.x; it < kHaloZ * kHaloY * kHaloX * CGC; it += kConvThreads) {
      const int h = it / CGC, cg = it - h * CGC;
      const int hx = h % kHaloX, hy = (h / kHaloX) % kHaloY, hz = h / (kHaloX * kHaloY);
      const bf16x8 v =
          load_in(p.in, c0 + cg, z0 + hz - 1, y0 + hy - 1, x0 + hx - 1, p.nz, p.ny, p.nx);
      halo[((hz * kHaloY + hy) * CGC + cg) * kHaloX + hx] = __builtin_bit_cast(u32x4, v);
    }
    __syncthreads();
    for (int q0 = 0; q0 < nq; q0 += 4) {
      const int q = q0 + g;
      bf16x8 aw = zero8(), bx[kTileY];
      if (q < nq) {
        const int tap = q / CGC, cg = q - tap * CGC;
        int dz, dy, dx;
        tap_offset(tap, dz, dy, dx);
        aw = ld8(p.w + (size_t)(cbase + j) * wrow + (size_t)(tap * CG + c0 + cg) * 8);
        const int base = ((wave + dz + 1) * kHaloY + dy + 1) * CGC + cg;
#pragma unroll
        for (int t = 0; t < kTileY; ++t)
          bx[t] = __builtin_bit_cast(bf16x8, halo[(base + t * CGC) * kHaloX + j + dx + 1]);
      } else {
#pragma unroll
        for (int t = 0; t < kTileY; ++t) bx[t] = zero8();
      }
#pragma unroll
      for (int t = 0; t < kTileY; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw, bx[t], acc[t], 0, 0, 0);
    }
  }
  const int x = x0 + j, z = z0 + wave;
#pragma unroll
  for (int t = 0; t < kTileY; ++t) {
    const int y = y0 + t;
    if (x < p.nx && y < p.ny && z < p.nz)
      conv_store<EPI>(p, N, ((size_t)z * p.ny + y) * p.nx + x, cbase + 4 * g, acc[t]);
  }
}

// Weight gradient of one tap (blockIdx.y): dW[o][tap][i] += sum_v dy[v][o] x[v + off][i]
// over the voxel chunks of this workgroup; the tiles go through LDS
// transposed ([channel][voxel]) so each lane reads 8 consecutive voxels of
// one channel as one 16-byte operand.  With more than 4 16x16 (o, i) tiles
// the waves share the tiles round-robin over one chunk at a time (R = 1).
// With at most 4 tiles (the full-resolution layers) R = 4 chunks are staged
// together and wave w multiplies every tile over chunk w of them; the four
// partial sums of a tile are added in chunk order at the end.  Each workgroup stores its sums in its own slab of the FP32
// partial buffer (every element of the slab, zeros where it saw no voxel),
// which k_sum_slabs adds up in workgroup order (deterministic).
struct WgradArgs {
  ConvIn in;
  const uint16_t* dy;   // BF16 [N][cout_pad]
  float* dw;            // FP32 partial slabs [gridDim.x][cout][27][cin_real]
  int cin_real;         // real input channels (the packed input may carry zero padding)
  int cout, cout_pad;
  int nz, ny, nx;
  int chunks;           // chunks of kWgradChunk voxels per workgroup
};

// chunks staged together for a layer with `tiles` 16x16 (o, i) tiles
__host__ __device__ constexpr int wgrad_group(int tiles) { return tiles <= 4 ? 4 : 1; }
// LDS row pitch (elements) of R chunks: 16-byte aligned rows
__host__ __device__ constexpr int wgrad_pitch(int R) { return kWgradChunk * R + 8; }

// Stage CH voxels x (8 ngroups) channels, read channels last by load(voxel,
// group), into dst[channel][voxel] (row pitch `pitch` elements, even): each
// thread takes two neighbouring voxels of one channel group and stores, per
// channel, their two 2-byte elements as one 4-byte word.
template <typename Load>
__device__ __forceinline__ void stage_pairs(uint16_t* dst, int pitch, int CH, int ngroups,
                                            Load load) {
  for (int it = threadIdx.x; it < (CH / 2) * ngroups; it += kConvThreads) {
    const int vp = it / ngroups, cg = it - vp * ngroups;
    const u32x4 a = __builtin_bit_cast(u32x4, load(2 * vp, cg));
    const u32x4 b = __builtin_bit_cast(u32x4, load(2 * vp + 1, cg));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t* row = reinterpret_cast<uint32_t*>(dst + (size_t)(cg * 8 + 2 * e) * pitch + 2 * vp);
      row[0] = (a[e] & 0xffffu) | (b[e] << 16);                              // channel 2e
      row[pitch / 2] = (a[e] >> 16) | (b[e] & 0xffff0000u);                  // channel 2e + 1
    }
  }
}

template <int R>
__global__ __launch_bounds__(kConvThreads) void k_conv3_wgrad(WgradArgs p) {
  extern __shared__ __align__(16) uint16_t smem[];
  constexpr int PITCH = wgrad_pitch(R);
  constexpr int CH = kWgradChunk * R;   // voxels staged at once
  const int cin = p.in.ca + p.in.cb;
  const int cit = (cin + 15) >> 4;          // input-channel tiles (x tile rows padded to 16)
  const int cot = p.cout_pad >> 4;
  const int ntiles = cot * cit;
  uint16_t* dyT = smem;                             // [cout_pad][PITCH]
  uint16_t* xT = smem + (size_t)p.cout_pad * PITCH;  // [cit * 16][PITCH]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  const int tap = blockIdx.y;
  int dz, dy, dx;
  tap_offset(tap, dz, dy, dx);
  const int N = p.nz * p.ny * p.nx;
  f32x4 acc[kWgradMaxTiles];
#pragma unroll
  for (int k = 0; k < kWgradMaxTiles; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  // zero the padding rows of the x tile once (channels cin .. cit*16)
  for (int r = cin + (threadIdx.x >> 6); r < cit * 16; r += 4)
    for (int c = lane; c < PITCH; c += 64) xT[(size_t)r * PITCH + c] = 0;
  const int cgo = p.cout_pad >> 3, cgi = cin >> 3;
  const int vend = ((int)blockIdx.x + 1) * p.chunks * kWgradChunk;   // this workgroup's range
  for (int ch = 0; ch < p.chunks; ch += R) {
    const int v0 = ((int)blockIdx.x * p.chunks + ch) * kWgradChunk;
    if (v0 >= N) break;
    __syncthreads();
    stage_pairs(dyT, PITCH, CH, cgo, [&](int vv, int cg) {
      const int v = v0 + vv;
      return v < N && v < vend ? ld8(p.dy + (size_t)v * p.cout_pad + cg * 8) : zero8();
    });
    stage_pairs(xT, PITCH, CH, cgi, [&](int vv, int cg) {
      const int v = v0 + vv;
      bf16x8 val = zero8();
      if (v < N && v < vend) {
        const int x = v % p.nx, y = (v / p.nx) % p.ny, z = v / (p.nx * p.ny);
        val = load_in(p.in, cg, z + dz, y + dy, x + dx, p.nz, p.ny, p.nx);
      }
      return val;
    });
    __syncthreads();
    if constexpr (R == 1) {
#pragma unroll
      for (int k = 0; k < kWgradMaxTiles; ++k) {
        const int t = wave + 4 * k;
        if (t < ntiles) {
          const int to = t / cit, ti = t - to * cit;
#pragma unroll
          for (int kk = 0; kk < kWgradChunk; kk += 32) {
            const bf16x8 a = ld8(dyT + (size_t)(to * 16 + j) * PITCH + kk + 8 * g);
            const bf16x8 b = ld8(xT + (size_t)(ti * 16 + j) * PITCH + kk + 8 * g);
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
          }
        }
      }
    } else {
      // ntiles <= 4: wave w takes every tile over chunk w
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < ntiles) {
          const int to = k / cit, ti = k - to * cit;
#pragma unroll
          for (int kk = 0; kk < kWgradChunk; kk += 32) {
            const int k0 = wave * kWgradChunk + kk + 8 * g;
            const bf16x8 a = ld8(dyT + (size_t)(to * 16 + j) * PITCH + k0);
            const bf16x8 b = ld8(xT + (size_t)(ti * 16 + j) * PITCH + k0);
            acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
          }
        }
      }
    }
  }
  float* slab = p.dw + (size_t)blockIdx.x * p.cout * 27 * p.cin_real;
  auto store_tile = [&](int t, const f32x4& r) {
    const int to = t / cit, ti = t - to * cit;
    const int i = ti * 16 + j;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int o = to * 16 + 4 * g + e;
      if (o < p.cout && i < p.cin_real) slab[((size_t)o * 27 + tap) * p.cin_real + i] = r[e];
    }
  };
  if constexpr (R == 1) {
#pragma unroll
    for (int k = 0; k < kWgradMaxTiles; ++k) {
      const int t = wave + 4 * k;
      if (t < ntiles) store_tile(t, acc[k]);
    }
  } else {
    // the four partial sums of each tile, added in chunk order: wave t < ntiles
    // stores tile t
    __syncthreads();   // the last chunk's tiles are read; smem is reused
    f32x4* part = reinterpret_cast<f32x4*>(smem);   // [wave][tile][lane]
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < ntiles) part[(wave * 4 + k) * 64 + lane] = acc[k];
    __syncthreads();
    if (wave < ntiles) {
      f32x4 r = part[wave * 64 + lane];
      for (int q = 1; q < 4; ++q) r += part[(q * 4 + wave) * 64 + lane];
      store_tile(wave, r);
    }
  }
}

// Partial bias gradients: slab b (this workgroup) of part receives
// sum_v dy[v][o] over the workgroup's voxels (BF16 dy, FP32 sums), the lanes
// of one channel added in lane order; k_sum_slabs adds the slabs up.
__global__ __launch_bounds__(kConvThreads) void k_bias_grad(const uint16_t* __restrict__ dy,
                                                            int N, int cout, int cout_pad,
                                                            float* __restrict__ part) {
  __shared__ float red[kConvThreads];
  const int c = threadIdx.x % cout_pad;
  const int lanes_per_voxel = kConvThreads / cout_pad;   // cout_pad divides 256
  const int sub = threadIdx.x / cout_pad;
  float s = 0.0f;
  for (int v = (int)blockIdx.x * lanes_per_voxel + sub; v < N; v += (int)gridDim.x * lanes_per_voxel)
    s += bf2f(dy[(size_t)v * cout_pad + c]);
  red[threadIdx.x] = s;
  __syncthreads();
  if ((int)threadIdx.x < cout) {
    float t = 0.0f;
    for (int k = 0; k < lanes_per_voxel; ++k) t += red[k * cout_pad + threadIdx.x];
    part[(size_t)blockIdx.x * cout + threadIdx.x] = t;
  }
}

// dst[e] += sum_b part[b][e] over the n_slab slabs of n elements, in slab
// order (the fixed-order end of the weight and bias gradients).
__global__ void k_sum_slabs(const float* __restrict__ part, int n_slab, size_t n,
                            float* __restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  // 16 slabs' loads in flight at a time; the additions keep slab order
  float t = 0.0f;
  int b = 0;
  for (; b + 16 <= n_slab; b += 16) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = part[(size_t)(b + k) * n + e];
#pragma unroll
    for (int k = 0; k < 16; ++k) t += v[k];
  }
  for (; b < n_slab; ++b) t += part[(size_t)b * n + e];
  dst[e] += t;
}

// Average over 2x2x2 blocks (BF16 in and out, FP32 sums); one thread per
// coarse voxel and 8-channel group.
__global__ void k_pool2(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int nz,
                        int ny, int nx, int C) {
  const int hz = nz >> 1, hy = ny >> 1, hx = nx >> 1;
  const int cg = C >> 3;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)hz * hy * hx * cg) return;
  const int g = (int)(id % cg);
  const size_t cv = id / cg;
  const int x = (int)(cv % hx), y = (int)((cv / hx) % hy), z = (int)(cv / ((size_t)hx * hy));
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < 8; ++d) {
    const size_t v = ((size_t)(2 * z + (d >> 2)) * ny + 2 * y + ((d >> 1) & 1)) * nx + 2 * x + (d & 1);
    const u32x4 w4 = *reinterpret_cast<const u32x4*>(in + v * C + g * 8);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      s[2 * e] += bf2f((uint16_t)(w4[e] & 0xffffu));
      s[2 * e + 1] += bf2f((uint16_t)(w4[e] >> 16));
    }
  }
  u32x4 o;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    o[e] = (uint32_t)f2bf(0.125f * s[2 * e]) | ((uint32_t)f2bf(0.125f * s[2 * e + 1]) << 16);
  *reinterpret_cast<u32x4*>(out + cv * C + g * 8) = o;
}

// fine[v][c] += coarse[v / 2][c] / 8 (adjoint of the 2x2x2 average), FP32.
__global__ void k_pool2_bwd_add(const float* __restrict__ coarse, float* __restrict__ fine, int nz,
                                int ny, int nx, int C) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nz * ny * nx * C;
  if (id >= n) return;
  const int c = (int)(id % C);
  const size_t v = id / C;
  const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((size_t)nx * ny));
  const size_t cv = ((size_t)(z >> 1) * (ny >> 1) + (y >> 1)) * (nx >> 1) + (x >> 1);
  fine[id] += 0.125f * coarse[cv * C + c];
}

// coarse[u][c] = sum of the 8 fine voxels of block u of dx[v][c] (c < ca), the
// adjoint of nearest-neighbour upsampling; dx has cin channels per voxel.
__global__ void k_up2_bwd(const float* __restrict__ dx, int cin, int ca, float* __restrict__ coarse,
                          int nz, int ny, int nx) {
  const int hz = nz >> 1, hy = ny >> 1, hx = nx >> 1;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (size_t)hz * hy * hx * ca) return;
  const int c = (int)(id % ca);
  const size_t cv = id / ca;
  const int x = (int)(cv % hx), y = (int)((cv / hx) % hy), z = (int)(cv / ((size_t)hx * hy));
  float s = 0.0f;
  for (int d = 0; d < 8; ++d) {
    const size_t v = ((size_t)(2 * z + (d >> 2)) * ny + 2 * y + ((d >> 1) & 1)) * nx + 2 * x + (d & 1);
    s += dx[v * cin + c];
  }
  coarse[id] = s;
}

// skip[v][c] = dx[v][ca + c] (the skip-branch part of a concatenated input gradient).
__global__ void k_take_skip(const float* __restrict__ dx, int cin, int ca, float* __restrict__ skip,
                            size_t N) {
  const int cb = cin - ca;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * cb) return;
  const size_t v = id / cb;
  skip[id] = dx[v * cin + ca + (id - v * cb)];
}

// dy_pre = dy * leaky'(.), the derivative read from the sign of the BF16
// activation output y; BF16 result.
__global__ void k_leaky_bwd(const uint16_t* __restrict__ y, const float* __restrict__ dy,
                            uint16_t* __restrict__ out, size_t n, float slope) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const float d = dy[id];
  out[id] = f2bf(bf2f(y[id]) > 0.0f ? d : slope * d);
}

// Site-major FP32 [C][N] -> BF16 channels last [N][cpad] (zero padding).
__global__ void k_to_channels_last(const float* __restrict__ in, int C, int cpad, size_t N,
                                   uint16_t* __restrict__ out) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= N * cpad) return;
  const size_t v = id / cpad;
  const int c = (int)(id - v * cpad);
  out[id] = c < C ? f2bf(in[(size_t)c * N + v]) : (uint16_t)0;
}

// Mean squared error over C x N values: per-block FP64 partial sums and the
// BF16 gradient 2 (o - t) / (C N) channels last [N][cpad] (zero padding).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out,
                                             const float* __restrict__ target, int C, int cpad,
                                             size_t N, uint16_t* __restrict__ grad,
                                             double* __restrict__ partials) {
  __shared__ double red[4];
  const double scale = 2.0 / ((double)C * (double)N);
  double s = 0.0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < N * cpad;
       id += (size_t)gridDim.x * blockDim.x) {
    const size_t v = id / cpad;
    const int c = (int)(id - v * cpad);
    float gval = 0.0f;
    if (c < C) {
      const double d = (double)out[(size_t)c * N + v] - (double)target[(size_t)c * N + v];
      s += d * d;
      gval = (float)(scale * d);
    }
    grad[id] = f2bf(gval);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_partials(const double* __restrict__ partials, int n, double scale,
                               double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += partials[i];
  *out = s * scale;
}

// FP32 master weights W[cout][27][cin] -> BF16 packed [cout_pad][27][cin_pad]
// (forward) and flipped [cin_pad16][27][cout_pad] with tap k -> 26 - k
// (backward data: the transposed convolution is a convolution with these).
__global__ void k_pack_weights(const float* __restrict__ W, int cout, int cin, int cout_pad,
                               int cin_pad, int cin_pad16, uint16_t* __restrict__ wp,
                               uint16_t* __restrict__ wf) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nfwd = (size_t)cout_pad * 27 * cin_pad;
  const size_t nflip = wf ? (size_t)cin_pad16 * 27 * cout_pad : 0;
  if (id < nfwd) {
    const int i = (int)(id % cin_pad);
    const int k = (int)((id / cin_pad) % 27);
    const int o = (int)(id / ((size_t)cin_pad * 27));
    wp[id] = (o < cout && i < cin) ? f2bf(W[((size_t)o * 27 + k) * cin + i]) : (uint16_t)0;
  } else if (id < nfwd + nflip) {
    const size_t f = id - nfwd;
    const int o = (int)(f % cout_pad);
    const int k = (int)((f / cout_pad) % 27);
    const int i = (int)(f / ((size_t)cout_pad * 27));
    wf[f] = (o < cout && i < cin) ? f2bf(W[((size_t)o * 27 + (26 - k)) * cin + i]) : (uint16_t)0;
  }
}

// Global gradient norm for clipping: per-block FP64 sums of squares (fixed
// block count and order), then one block forms scale = min(1, clip / |g|).
constexpr int kNormBlocks = 256;

__global__ __launch_bounds__(256) void k_sumsq(const float* __restrict__ g, size_t n,
                                               double* __restrict__ partials) {
  __shared__ double red[4];
  double s = 0.0;
  for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < n;
       id += (size_t)gridDim.x * blockDim.x)
    s += (double)g[id] * (double)g[id];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_clip_scale(double* __restrict__ partials, int nb, double clip) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += partials[i];
  const double norm = sqrt(s);
  partials[nb] = norm;                                   // |g| before clipping
  partials[nb + 1] = norm > clip ? clip / norm : 1.0;    // scale applied to g
}

// Adam with bias correction, FP32 master parameters; the gradient is first
// multiplied by *scale when scale is not null (global-norm clipping).
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, size_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, const double* __restrict__ scale) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const float gr = scale ? (float)((double)grad[id] * *scale) : grad[id];
  const float mm = b1 * m[id] + (1.0f - b1) * gr;
  const float vv = b2 * v[id] + (1.0f - b2) * gr * gr;
  m[id] = mm;
  v[id] = vv;
  theta[id] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_fill_f32(float* __restrict__ p, size_t n, float value) {
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id < n) p[id] = value;
}

}  // namespace net
}  // namespace rism
