// LDS-staged Stockham mixed-radix FFT passes for gfx950.
//
// The solver's transforms are the half-integer-shifted DFTs of the section
// "Numerical procedure" (k at half-integer points, r at integer points):
//   forward  X_j = sum_a x_a exp(-2 pi i (j + 1/2) a / n)
//   inverse  x_a = sum_j X_j exp(+2 pi i (j + 1/2) a / n)      (unnormalised)
// per axis.  exp(-2 pi i (j+1/2) a/n) = exp(-i pi a/n) exp(-2 pi i j a/n), so a
// forward axis pass multiplies by exp(-i pi a/n) on load and runs a plain DFT;
// an inverse pass runs the plain inverse DFT and multiplies by exp(+i pi a/n)
// on store.  The 1/N and dV factors are folded into the k-space tables.
//
// One workgroup owns a tile of whole lines: for the x axis several contiguous
// rows, for the y and z axes a run of consecutive x columns (so each row of the
// tile is a coalesced 128 B segment).  The tile is loaded into LDS, transformed
// by Stockham autosort passes (radix 2/3/4/5/8/16, ping-pong between two LDS
// buffers, natural-order output) and written back in place.  The bulk
// iterations run it on float2; the periodic FP64 anchor evaluations on double2.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace rism {

constexpr int kFftThreads = 256;
constexpr int kFftTileBytes = 32768;  // bytes per LDS ping-pong buffer
constexpr int kFftMaxN = 512;

template <typename C>
constexpr int fft_tile_elems() { return kFftTileBytes / (int)sizeof(C); }

// Radix-R DFT in registers: X_q = sum_r v_r exp(sgn 2 pi i q r / R).
template <int R, typename C, typename S>
struct Dft;

template <typename C, typename S>
struct Dft<2, C, S> {
  __device__ static inline void run(C* v, S) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename C, typename S>
struct Dft<4, C, S> {
  __device__ static inline void run(C* v, S sgn) {
    C t0 = cadd(v[0], v[2]);
    C t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]);
    C t3 = cmul_i(csub(v[1], v[3]), sgn);   // sgn * i * (v1 - v3)
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <typename C, typename S>
struct Dft<8, C, S> {
  __device__ static inline void run(C* v, S sgn) {
    const S h = S(0.70710678118654752440);   // sqrt(1/2)
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, C, S>::run(e, sgn);
    Dft<4, C, S>::run(o, sgn);
    // o_q *= exp(sgn 2 pi i q / 8)
    const C o1 = cmul(o[1], make_c(h, sgn * h));
    const C o2 = cmul_i(o[2], sgn);
    const C o3 = cmul(o[3], make_c(-h, sgn * h));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// 16 = 2 x 8: the even and odd halves by radix 8, then the twiddles
// exp(sgn 2 pi i q / 16), q < 8, and the final radix-2 step.
template <typename C, typename S>
struct Dft<16, C, S> {
  __device__ static inline void run(C* v, S sgn) {
    const S h = S(0.70710678118654752440);    // cos(pi/4) = sin(pi/4)
    const S c1 = S(0.92387953251128675613);   // cos(pi/8)
    const S s1 = S(0.38268343236508977173);   // sin(pi/8)
    C e[8], o[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      e[r] = v[2 * r];
      o[r] = v[2 * r + 1];
    }
    Dft<8, C, S>::run(e, sgn);
    Dft<8, C, S>::run(o, sgn);
    o[1] = cmul(o[1], make_c(c1, sgn * s1));
    o[2] = cmul(o[2], make_c(h, sgn * h));
    o[3] = cmul(o[3], make_c(s1, sgn * c1));
    o[4] = cmul_i(o[4], sgn);
    o[5] = cmul(o[5], make_c(-s1, sgn * c1));
    o[6] = cmul(o[6], make_c(-h, sgn * h));
    o[7] = cmul(o[7], make_c(-c1, sgn * s1));
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      v[q] = cadd(e[q], o[q]);
      v[q + 8] = csub(e[q], o[q]);
    }
  }
};

template <typename C, typename S>
struct Dft<3, C, S> {
  __device__ static inline void run(C* v, S sgn) {
    const S c = S(-0.5);
    const S s = S(0.86602540378443864676);   // sin(2 pi / 3)
    C a = cadd(v[1], v[2]);
    C b = csub(v[1], v[2]);
    C m = make_c(v[0].x + c * a.x, v[0].y + c * a.y);
    C ib = cmul_i(b, sgn * s);                 // sgn * i * s * (v1 - v2)
    v[0] = cadd(v[0], a);
    v[1] = cadd(m, ib);
    v[2] = csub(m, ib);
  }
};

template <typename C, typename S>
struct Dft<5, C, S> {
  __device__ static inline void run(C* v, S sgn) {
    const S c1 = S(0.30901699437494742410);    // cos(2 pi / 5)
    const S c2 = S(-0.80901699437494742410);   // cos(4 pi / 5)
    const S s1 = S(0.95105651629515357212);    // sin(2 pi / 5)
    const S s2 = S(0.58778525229247312917);    // sin(4 pi / 5)
    C a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    C a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    C m1 = make_c(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
    C m2 = make_c(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
    C n1 = make_c(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
    C n2 = make_c(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
    C in1 = cmul_i(n1, sgn);
    C in2 = cmul_i(n2, sgn);
    v[0] = make_c(v[0].x + a1.x + a2.x, v[0].y + a1.y + a2.y);
    v[1] = cadd(m1, in1);
    v[4] = csub(m1, in1);
    v[2] = cadd(m2, in2);
    v[3] = csub(m2, in2);
  }
};

// One Stockham pass of radix R over `nlines` lines of length n in LDS.
// Ns is the product of the radices already applied.  tw2[m] = exp(-2 pi i m / (2n)).
template <int R, typename C, typename S>
__device__ inline void stockham_pass(const C* __restrict__ src, C* __restrict__ dst, int nlines,
                                     int n, int Ns, const C* tw2, S sgn) {
  const int nb = n / R;
  const int step2 = (2 * n) / (Ns * R);   // exp(-2 pi i r k/(Ns R)) = tw2[r k step2]
  const int two_n = 2 * n;
  for (int t = threadIdx.x; t < nlines * nb; t += blockDim.x) {
    const int b = t / nb;
    const int j = t - b * nb;
    const C* s = src + b * n;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = tw2[(r * k * step2) % two_n];
        v[r] = (sgn < S(0)) ? cmul(v[r], w) : cmulc(v[r], w);
      }
    }
    Dft<R, C, S>::run(v, sgn);
    C* d = dst + b * n + (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[r * Ns] = v[r];
  }
}

// Runs all passes of `plan`; returns the LDS buffer that holds the result.
template <typename C, typename S>
__device__ inline C* lds_fft(C* bufA, C* bufB, int nlines, const AxisPlan& plan, const C* tw2,
                             S sgn) {
  C* src = bufA;
  C* dst = bufB;
  int Ns = 1;
  for (int p = 0; p < plan.npass; ++p) {
    const int R = plan.radix[p];
    switch (R) {
      case 2: stockham_pass<2>(src, dst, nlines, plan.n, Ns, tw2, sgn); break;
      case 3: stockham_pass<3>(src, dst, nlines, plan.n, Ns, tw2, sgn); break;
      case 4: stockham_pass<4>(src, dst, nlines, plan.n, Ns, tw2, sgn); break;
      case 5: stockham_pass<5>(src, dst, nlines, plan.n, Ns, tw2, sgn); break;
      default: stockham_pass<8>(src, dst, nlines, plan.n, Ns, tw2, sgn); break;
    }
    __syncthreads();
    Ns *= R;
    C* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Lines per workgroup for an axis pass (host helper).
template <typename C>
inline int fft_lines_per_block(int axis, int n, int nx) {
  const int tile = fft_tile_elems<C>();
  if (axis == 0) {
    const int l = tile / n;
    return l < 1 ? 1 : l;
  }
  int l = tile / n;
  if (l > 16) l = 16;
  if (l > nx) l = nx;
  return l;
}

// Axis pass over complex grids data[npair][nz][ny][nx] (C = float2 or double2).
// axis 0 = x (rows), 1 = y, 2 = z.  forward != 0: shifted forward transform;
// otherwise shifted inverse (unnormalised).  `lines` = lines per workgroup.
template <typename C>
__global__ __launch_bounds__(kFftThreads) void k_fft_axis(
    C* __restrict__ data, int nx, int ny, int nz, int npair, int axis, AxisPlan plan,
    const C* __restrict__ tw2_g, int forward, int lines, const int* __restrict__ done) {
  using S = typename ScalarOf<C>::type;
  constexpr int TILE = fft_tile_elems<C>();
  if (done && skip_iteration<std::is_same<C, double2>::value>(*done)) return;
  __shared__ C lds[2 * TILE + 2 * kFftMaxN];
  C* bufA = lds;
  C* bufB = lds + TILE;
  C* tw2 = lds + 2 * TILE;
  const int n = plan.n;
  for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) tw2[i] = tw2_g[i];

  // Tile geometry: element (b, i) of the tile lives at base + b * bstride + i * istride.
  size_t base;
  int nl;
  size_t bstride, istride;
  if (axis == 0) {
    const size_t rows = (size_t)npair * nz * ny;
    const size_t row0 = (size_t)blockIdx.x * lines;
    if (row0 >= rows) return;
    nl = (int)((rows - row0) < (size_t)lines ? (rows - row0) : (size_t)lines);
    base = row0 * nx;
    bstride = nx;
    istride = 1;
  } else {
    const int tiles_x = (nx + lines - 1) / lines;
    const int outer = blockIdx.x / tiles_x;   // (p, z) for y; (p, y) for z
    const int x0 = (blockIdx.x - outer * tiles_x) * lines;
    nl = (nx - x0) < lines ? (nx - x0) : lines;
    bstride = 1;
    if (axis == 1) {
      base = (size_t)outer * ny * nx + x0;
      istride = nx;
    } else {
      const int p = outer / ny;
      const int y = outer - p * ny;
      base = ((size_t)p * nz * ny + y) * nx + x0;
      istride = (size_t)ny * nx;
    }
  }
  __syncthreads();

  const int total = nl * n;
  for (int f = threadIdx.x; f < total; f += blockDim.x) {
    int b, i;
    if (axis == 0) { b = f / n; i = f - b * n; }
    else { i = f / nl; b = f - i * nl; }
    C v = data[base + b * bstride + i * istride];
    if (forward) v = cmul(v, tw2[i]);              // exp(-i pi i / n)
    bufA[b * n + i] = v;
  }
  __syncthreads();
  C* res = lds_fft(bufA, bufB, nl, plan, tw2, forward ? S(-1) : S(1));
  for (int f = threadIdx.x; f < total; f += blockDim.x) {
    int b, i;
    if (axis == 0) { b = f / n; i = f - b * n; }
    else { i = f / nl; b = f - i * nl; }
    C v = res[b * n + i];
    if (!forward) v = cmulc(v, tw2[i]);            // exp(+i pi i / n)
    data[base + b * bstride + i * istride] = v;
  }
}

// ---------------------------------------------------------------------------
// Fixed-size passes for the common axis lengths.  The radix plan, tile shape
// and index arithmetic are compile-time constants; every thread issues all its
// global loads before touching LDS (memory-level parallelism), and the radix
// passes run in place in one LDS tile (each thread holds its butterfly inputs
// in registers across the barrier), which halves the LDS footprint of the
// ping-pong kernel and doubles its occupancy.
// ---------------------------------------------------------------------------
template <int N> struct FixedPlan { static constexpr int n = 0; };
template <> struct FixedPlan<32>  { static constexpr int n = 2; static constexpr int r[4] = {8, 4, 1, 1}; };
template <> struct FixedPlan<64>  { static constexpr int n = 2; static constexpr int r[4] = {8, 8, 1, 1}; };
template <> struct FixedPlan<96>  { static constexpr int n = 3; static constexpr int r[4] = {8, 4, 3, 1}; };
template <> struct FixedPlan<128> { static constexpr int n = 3; static constexpr int r[4] = {8, 4, 4, 1}; };
template <> struct FixedPlan<192> { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 3, 1}; };
template <> struct FixedPlan<256> { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 4, 1}; };
template <> struct FixedPlan<512> { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 8, 1}; };

// Plans with a radix-16 first pass (two passes instead of three at 128 and
// 256 points), for kernels whose tiles hold many lines.
template <int N> struct WidePlan : FixedPlan<N> {};
template <> struct WidePlan<128> { static constexpr int n = 2; static constexpr int r[4] = {16, 8, 1, 1}; };
template <> struct WidePlan<256> { static constexpr int n = 2; static constexpr int r[4] = {16, 16, 1, 1}; };

inline bool fixed_fft_size(int n) {
  return n == 32 || n == 64 || n == 96 || n == 128 || n == 192 || n == 256 || n == 512;
}

template <typename C> constexpr int fixed_tile() { return sizeof(C) == 8 ? 4096 : 2048; }

template <typename C, int N, int AXIS>
constexpr int fixed_lines() {
  return AXIS == 0 ? (fixed_tile<C>() / N < 1 ? 1 : fixed_tile<C>() / N)
                   : (fixed_tile<C>() / N > 32 ? 32 : fixed_tile<C>() / N);
}

// LDS layout of a tile: element i of line b lives at b * PITCH + i + (i >> 3).
// The skew of one slot every 8 elements makes the stride-R writes of the first
// Stockham pass conflict-free, and the odd pitch does the same for the
// transposed (one lane per line) accesses of the y and z passes.
template <int N> struct Lds {
  static constexpr int PITCH = N + N / 8 + 1;
  __device__ static inline int at(int b, int i) { return b * PITCH + i + (i >> 3); }
};

template <int R, int NS, int N, int LINES, typename C, typename S>
__device__ inline void pass_inplace(C* buf, int nl, const C* tw2, S sgn) {
  constexpr int NB = N / R;
  constexpr int MAXB = (LINES * NB + kFftThreads - 1) / kFftThreads;
  constexpr int STEP2 = (2 * N) / (NS * R);
  const int nbf = nl * NB;
  C v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = threadIdx.x + q * kFftThreads;
    if (t < nbf) {
      const int b = t / NB;
      const int j = t - b * NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[Lds<N>::at(b, j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int t = threadIdx.x + q * kFftThreads;
    if (t < nbf) {
      const int b = t / NB;
      const int j = t - b * NB;
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const C w = tw2[(r * k * STEP2) % (2 * N)];
          v[q][r] = (sgn < S(0)) ? cmul(v[q][r], w) : cmulc(v[q][r], w);
        }
      }
      Dft<R, C, S>::run(v[q], sgn);
      const int d0 = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[Lds<N>::at(b, d0 + r * NS)] = v[q][r];
    }
  }
  __syncthreads();
}

template <int P, int NS, int N, int LINES, typename PL = FixedPlan<N>, typename C, typename S>
__device__ inline void passes_from(C* buf, int nl, const C* tw2, S sgn) {
  if constexpr (P < PL::n) {
    constexpr int R = PL::r[P];
    pass_inplace<R, NS, N, LINES>(buf, nl, tw2, sgn);
    passes_from<P + 1, NS * R, N, LINES, PL>(buf, nl, tw2, sgn);
  }
}

// LINES (lines per workgroup) defaults to fixed_lines; the autotuner may pick
// another width for the y pass; it does not change the operations on a line.
template <typename C, int N, int AXIS, int LINES = fixed_lines<C, N, AXIS>()>
__global__ __launch_bounds__(kFftThreads) void k_fft_fixed(
    C* __restrict__ data, int nx, int ny, int nz, int npair, const C* __restrict__ tw2_g,
    int forward, const int* __restrict__ done, size_t bstride) {
  using S = typename ScalarOf<C>::type;
  // y and z tiles hold LINES whole lines: the radix-16 plans
  using Plan = typename std::conditional<AXIS != 0, WidePlan<N>, FixedPlan<N>>::type;
  constexpr int TILE = LINES * N;
  constexpr int EPT = (TILE + kFftThreads - 1) / kFftThreads;
  done = member_ptr(done, bstride);
  if (done && skip_iteration<std::is_same<C, double2>::value>(*done)) return;
  data = member_ptr(data, bstride);
  tw2_g = member_ptr(tw2_g, bstride);
  __shared__ C buf[LINES * Lds<N>::PITCH];
  __shared__ C tw2[2 * N];
  for (int i = threadIdx.x; i < 2 * N; i += kFftThreads) tw2[i] = tw2_g[i];

  size_t base;
  int nl;
  size_t istride;
  if (AXIS == 0) {
    const size_t rows = (size_t)npair * nz * ny;
    const size_t row0 = (size_t)blockIdx.x * LINES;
    if (row0 >= rows) return;
    nl = (int)((rows - row0) < (size_t)LINES ? (rows - row0) : (size_t)LINES);
    base = row0 * N;
    istride = 1;
  } else {
    const int tiles_x = (nx + LINES - 1) / LINES;
    const int outer = blockIdx.x / tiles_x;
    const int x0 = (blockIdx.x - outer * tiles_x) * LINES;
    nl = (nx - x0) < LINES ? (nx - x0) : LINES;
    if (AXIS == 1) {
      base = (size_t)outer * N * nx + x0;
      istride = nx;
    } else {
      const int p = outer / ny;
      const int y = outer - p * ny;
      base = ((size_t)p * N * ny + y) * nx + x0;
      istride = (size_t)ny * nx;
    }
  }
  const int total = nl * N;
  // FP32 y/z tiles of full width move neighbouring lines (x, x+1) as one
  // 16-byte vector: half the memory instructions, no runtime index division.
  constexpr bool kVec = std::is_same<C, float2>::value && AXIS != 0 && LINES % 2 == 0;
  const bool vec = kVec && nl == LINES;
  if constexpr (kVec) {
    if (vec) {
      constexpr int H = LINES / 2;
      constexpr int EPT2 = (H * N + kFftThreads - 1) / kFftThreads;
      float4 w4[EPT2];
#pragma unroll
      for (int e = 0; e < EPT2; ++e) {
        const int f = threadIdx.x + e * kFftThreads;
        if (f < H * N) {
          const int i = f / H, h = f - i * H;
          w4[e] = *reinterpret_cast<const float4*>(data + base + 2 * h + i * istride);
        }
      }
      __syncthreads();   // twiddles visible
#pragma unroll
      for (int e = 0; e < EPT2; ++e) {
        const int f = threadIdx.x + e * kFftThreads;
        if (f < H * N) {
          const int i = f / H, h = f - i * H;
          const C a = make_float2(w4[e].x, w4[e].y), b = make_float2(w4[e].z, w4[e].w);
          buf[Lds<N>::at(2 * h, i)] = forward ? cmul(a, tw2[i]) : a;
          buf[Lds<N>::at(2 * h + 1, i)] = forward ? cmul(b, tw2[i]) : b;
        }
      }
      __syncthreads();
      passes_from<0, 1, N, LINES, Plan>(buf, nl, tw2, forward ? S(-1) : S(1));
      for (int f = threadIdx.x; f < H * N; f += kFftThreads) {
        const int i = f / H, h = f - i * H;
        C a = buf[Lds<N>::at(2 * h, i)], b = buf[Lds<N>::at(2 * h + 1, i)];
        if (!forward) {
          a = cmulc(a, tw2[i]);
          b = cmulc(b, tw2[i]);
        }
        *reinterpret_cast<float4*>(data + base + 2 * h + i * istride) =
            make_float4(a.x, a.y, b.x, b.y);
      }
      return;
    }
  }
  C v[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int f = threadIdx.x + e * kFftThreads;
    if (f < total) {
      if (AXIS == 0) v[e] = data[base + f];
      else {
        const int i = f / nl, b = f - i * nl;
        v[e] = data[base + b + i * istride];
      }
    }
  }
  __syncthreads();   // twiddles visible
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int f = threadIdx.x + e * kFftThreads;
    if (f < total) {
      int b, i;
      if (AXIS == 0) { b = f / N; i = f - b * N; }
      else { i = f / nl; b = f - i * nl; }
      buf[Lds<N>::at(b, i)] = forward ? cmul(v[e], tw2[i]) : v[e];
    }
  }
  __syncthreads();
  passes_from<0, 1, N, LINES, Plan>(buf, nl, tw2, forward ? S(-1) : S(1));
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int f = threadIdx.x + e * kFftThreads;
    if (f < total) {
      int b, i;
      if (AXIS == 0) { b = f / N; i = f - b * N; }
      else { i = f / nl; b = f - i * nl; }
      C o = buf[Lds<N>::at(b, i)];
      if (!forward) o = cmulc(o, tw2[i]);
      if (AXIS == 0) data[base + f] = o;
      else data[base + b + i * istride] = o;
    }
  }
}

}  // namespace rism
