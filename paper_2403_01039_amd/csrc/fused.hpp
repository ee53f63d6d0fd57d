// Fused iteration kernels for grids whose x length has a fixed-size FFT plan:
//   k_update_fftx    MDIIS update + closure (steps 6 and 2) fused with the
//                    forward x-axis transform of step 3;
//   k_fftx_residual  inverse x-axis transform of step 5 fused with the
//                    residual (Eq 33) and the MDIIS Gram row.
// Each saves one full read and write of the packed spectra per iteration.
#pragma once

#include <type_traits>

#include "fft.hpp"
#include "iterate.hpp"

namespace rism {

template <bool ANCHOR>
using PrecC = typename std::conditional<ANCHOR, double2, float2>::type;

// LINES (x rows per workgroup) of both fused kernels defaults to fixed_lines;
// the autotuner may pick another count for the FP32 iterations.
template <bool ANCHOR, int N, int LINES = fixed_lines<PrecC<ANCHOR>, N, 0>(), int MM = kMaxDepth>
__global__ __launch_bounds__(kFftThreads) void k_update_fftx(
    const IterState* __restrict__ st, float* __restrict__ tau_hist,
    const float* __restrict__ res_hist, const float* __restrict__ w,
    const float* __restrict__ tau_ref, const float* __restrict__ tau_lo,
    const float* __restrict__ dref, float* __restrict__ dg_out, void* __restrict__ spec_v,
    int ny, int nz, int nv, int npair, int M, int kind, int order,
    const PrecC<ANCHOR>* __restrict__ tw2_g, size_t bstride) {
  using C = PrecC<ANCHOR>;
  using S = typename ScalarOf<C>::type;
  constexpr int Q = N / 4;
  st = member_ptr(st, bstride);
  if (skip_iteration<ANCHOR>(st->done)) return;
  tau_hist = member_ptr(tau_hist, bstride);
  res_hist = member_ptr(res_hist, bstride);
  w = member_ptr(w, bstride);
  tau_ref = member_ptr(tau_ref, bstride);
  tau_lo = member_ptr(tau_lo, bstride);
  dref = member_ptr(dref, bstride);
  dg_out = member_ptr(dg_out, bstride);
  spec_v = member_ptr(spec_v, bstride);
  tw2_g = member_ptr(tw2_g, bstride);
  __shared__ C buf[LINES * Lds<N>::PITCH];
  __shared__ C tw2[2 * N];
  for (int i = threadIdx.x; i < 2 * N; i += kFftThreads) tw2[i] = tw2_g[i];
  const size_t plane = (size_t)nz * ny;
  const size_t rows = (size_t)npair * plane;
  const size_t row0 = (size_t)blockIdx.x * LINES;
  if (row0 >= rows) return;
  const int nl = (int)((rows - row0) < (size_t)LINES ? (rows - row0) : (size_t)LINES);
  const size_t N3 = (size_t)N * plane;
  const UpdateCtl u = load_update_ctl(st, M);
  __syncthreads();
  for (int t = threadIdx.x; t < nl * Q; t += kFftThreads) {
    const int b = t / Q;
    const int i0 = (t - b * Q) * 4;
    const size_t row = row0 + b;
    const int p = (int)(row / plane);
    const size_t n = (row - (size_t)p * plane) * N + i0;
    double o64[2][4];
    float o32[2][4];
    update_points<ANCHOR, 4, MM>(u, tau_hist, res_hist, w, tau_ref, tau_lo, dref, dg_out, N3, nv,
                                 p, n, kind, order, o64, o32);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const C val = ANCHOR ? make_c((S)o64[0][v], (S)o64[1][v]) : make_c((S)o32[0][v], (S)o32[1][v]);
      buf[Lds<N>::at(b, i0 + v)] = cmul(val, tw2[i0 + v]);   // exp(-i pi a / n)
    }
  }
  __syncthreads();
  passes_from<0, 1, N, LINES>(buf, nl, tw2, S(-1));
  C* spec = static_cast<C*>(spec_v) + row0 * N;
  for (int f = threadIdx.x; f < nl * N; f += kFftThreads) {
    const int b = f / N, i = f - b * N;
    spec[f] = buf[Lds<N>::at(b, i)];
  }
}

// MM: compile-time bound on the history depth (the Gram accumulators held per
// thread); the launch picks the smallest instantiated bound >= M.
template <bool ANCHOR, int N, int LINES = fixed_lines<PrecC<ANCHOR>, N, 0>(), int MM = kMaxDepth>
__global__ __launch_bounds__(kFftThreads) void k_fftx_residual(
    const IterState* __restrict__ st, const void* __restrict__ spec_v,
    const float* __restrict__ w, float* __restrict__ tau_hist, float* __restrict__ res_hist,
    float* __restrict__ tau_ref, float* __restrict__ tau_lo, float* __restrict__ r_ref,
    float* __restrict__ dref, const float* __restrict__ dg, int ny, int nz, int nv, int npair,
    int M, int kind, int order,
    const PrecC<ANCHOR>* __restrict__ tw2_g, double* __restrict__ partials, GramW gw,
    size_t bstride) {
  using C = PrecC<ANCHOR>;
  using S = typename ScalarOf<C>::type;
  constexpr int Q = N / 4;
  st = member_ptr(st, bstride);
  if (skip_iteration<ANCHOR>(st->done)) return;
  spec_v = member_ptr(spec_v, bstride);
  w = member_ptr(w, bstride);
  tau_hist = member_ptr(tau_hist, bstride);
  res_hist = member_ptr(res_hist, bstride);
  tau_ref = member_ptr(tau_ref, bstride);
  tau_lo = member_ptr(tau_lo, bstride);
  r_ref = member_ptr(r_ref, bstride);
  dref = member_ptr(dref, bstride);
  dg = member_ptr(dg, bstride);
  tw2_g = member_ptr(tw2_g, bstride);
  partials = member_ptr(partials, bstride);
  __shared__ C buf[LINES * Lds<N>::PITCH];
  __shared__ C tw2[2 * N];
  __shared__ double red[(MM + 1) * (kFftThreads / 64)];
  for (int i = threadIdx.x; i < 2 * N; i += kFftThreads) tw2[i] = tw2_g[i];
  const size_t plane = (size_t)nz * ny;
  const size_t rows = (size_t)npair * plane;
  const size_t row0 = (size_t)blockIdx.x * LINES;
  const int nl = (int)((rows - row0) < (size_t)LINES ? (rows - row0) : (size_t)LINES);
  const size_t N3 = (size_t)N * plane;
  const int dest = st->dest;
  const unsigned mask = other_slots(st, M, dest);
  const C* spec = static_cast<const C*>(spec_v) + row0 * N;
  if constexpr (ANCHOR) {
    for (int f = threadIdx.x; f < nl * N; f += kFftThreads) {
      const int b = f / N, i = f - b * N;
      buf[Lds<N>::at(b, i)] = spec[f];
    }
  } else {
    // every load of the tile in flight before the first LDS store (the FP64
    // variant keeps the plain loop: staging its tile would spill)
    constexpr int EPT = (LINES * N + kFftThreads - 1) / kFftThreads;
    C v[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int f = threadIdx.x + e * kFftThreads;
      if (f < nl * N) v[e] = spec[f];
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int f = threadIdx.x + e * kFftThreads;
      if (f < nl * N) {
        const int b = f / N, i = f - b * N;
        buf[Lds<N>::at(b, i)] = v[e];
      }
    }
  }
  __syncthreads();
  passes_from<0, 1, N, LINES>(buf, nl, tw2, S(1));
  double acc[MM + 1];
#pragma unroll
  for (int i = 0; i <= MM; ++i) acc[i] = 0.0;
  for (int t = threadIdx.x; t < nl * Q; t += kFftThreads) {
    const int b = t / Q;
    const int i0 = (t - b * Q) * 4;
    const size_t row = row0 + b;
    const int p = (int)(row / plane);
    const size_t n = (row - (size_t)p * plane) * N + i0;
    float hre[4], him[4];
    double h64[2][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const C h = cmulc(buf[Lds<N>::at(b, i0 + v)], tw2[i0 + v]);   // exp(+i pi a / n)
      hre[v] = (float)h.x;
      him[v] = (float)h.y;
      h64[0][v] = (double)h.x;
      h64[1][v] = (double)h.y;
    }
    residual_points<ANCHOR, 4, MM>(hre, him, h64, w, tau_hist, res_hist, tau_ref, tau_lo, r_ref,
                                   dref, dg, N3, nv, p, n, dest, mask, kind, order, gw, acc);
  }
  write_partials<MM>(acc, M, partials, red);
}

}  // namespace rism

namespace rism {

// ---------------------------------------------------------------------------
// k_zcz: forward z transform + k-space contraction (Eq 13, Eq 32) + inverse z
// transform in one pass over the packed spectra.  A workgroup owns, for every
// site pair, the z-columns (x0..x0+B-1, y) and their mirror columns
// (nx-1-x, ny-1-y), so each k-point meets its partner -k on chip.  Requires an
// even ny (columns y < ny/2 pair with y' = ny-1-y >= ny/2).
// ---------------------------------------------------------------------------
template <typename C, int NZ, int NV>
constexpr int zcz_cols() {
  // largest B (<= 16) with the 2 * P * B columns of NZ in ~64 KB of LDS
  constexpr int P = (NV + 1) / 2;
  constexpr int per_col = 2 * P * Lds<NZ>::PITCH * (int)sizeof(C);
  return per_col * 16 <= 65536 ? 16 : per_col * 8 <= 65536 ? 8 : per_col * 4 <= 65536 ? 4 : 2;
}

// B (columns per side and workgroup) defaults to zcz_cols; the autotuner may
// pick another width; it does not change the operations on a column.
template <typename C, int NZ, int NV, bool WITHF, int B = zcz_cols<C, NZ, NV>()>
__global__ __launch_bounds__(kFftThreads) void k_zcz(
    C* __restrict__ spec, int nx, int ny, const C* __restrict__ tw2_g, double dkx, double dky,
    double dkz, const C* __restrict__ F, const typename ScalarOf<C>::type* __restrict__ chi,
    const typename ScalarOf<C>::type* __restrict__ qtab, double inv_dkt, int m_tab,
    const int* __restrict__ done, size_t bstride) {
  using S = typename ScalarOf<C>::type;
  constexpr int P = (NV + 1) / 2;
  constexpr int LINES = 2 * P * B;     // line l = (side * P + p) * B + b
  done = member_ptr(done, bstride);
  if (done && skip_iteration<std::is_same<C, double2>::value>(*done)) return;
  spec = member_ptr(spec, bstride);
  tw2_g = member_ptr(tw2_g, bstride);
  F = member_ptr(F, bstride);
  chi = member_ptr(chi, bstride);
  qtab = member_ptr(qtab, bstride);
  __shared__ C buf[LINES * Lds<NZ>::PITCH];
  __shared__ C tw2[2 * NZ];
  for (int i = threadIdx.x; i < 2 * NZ; i += kFftThreads) tw2[i] = tw2_g[i];
  const int tiles_x = (nx + B - 1) / B;
  const int tile = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int jy = tile / tiles_x;                       // 0 .. ny/2 - 1
  const int x0 = (tile - jy * tiles_x) * B;
  const int nb = (nx - x0) < B ? (nx - x0) : B;
  const int jy2 = ny - 1 - jy;
  const size_t N = (size_t)nx * ny * NZ;
  const size_t zs = (size_t)nx * ny;
  // element (l, z) <-> global address; side 1 columns run backwards in x
  auto addr = [&](int side, int p, int b, int z) -> size_t {
    const int x = side ? nx - 1 - (x0 + b) : x0 + b;
    return (size_t)p * N + (size_t)z * zs + (size_t)(side ? jy2 : jy) * nx + x;
  };
  const int total = 2 * P * nb * NZ;
  // FP32 tiles of full width move column pairs as 16-byte vectors: on side 0
  // the pair (b, b+1) sits at x0+b, x0+b+1; on side 1, where columns run
  // backwards in x, at nx-2-x0-b (column b+1) and nx-1-x0-b (column b).
  constexpr bool kVec = std::is_same<C, float2>::value && B % 2 == 0;
  constexpr int H = B / 2;
  auto pair_addr = [&](int side, int p, int h, int z) -> size_t {
    const int x = side ? nx - 2 - x0 - 2 * h : x0 + 2 * h;
    return (size_t)p * N + (size_t)z * zs + (size_t)(side ? jy2 : jy) * nx + x;
  };
  const bool vec = kVec && nb == B;
  if constexpr (kVec) {
   if (vec) {
    constexpr int TOT = 2 * P * H * NZ;
    constexpr int EPT = (TOT + kFftThreads - 1) / kFftThreads;
    float4 v[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int f = threadIdx.x + e * kFftThreads;
      if (f < TOT) {
        const int h = f % H;
        const int r = f / H;
        const int z = r % NZ;
        const int sp = r / NZ;
        const int side = sp / P, p = sp - side * P;
        v[e] = *reinterpret_cast<const float4*>(spec + pair_addr(side, p, h, z));
      }
    }
    __syncthreads();   // twiddles visible
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int f = threadIdx.x + e * kFftThreads;
      if (f < TOT) {
        const int h = f % H;
        const int r = f / H;
        const int z = r % NZ;
        const int sp = r / NZ;
        const int side = sp / P;
        const float2 lo = make_float2(v[e].x, v[e].y), hi = make_float2(v[e].z, v[e].w);
        buf[Lds<NZ>::at(sp * B + 2 * h, z)] = cmul(side ? hi : lo, tw2[z]);
        buf[Lds<NZ>::at(sp * B + 2 * h + 1, z)] = cmul(side ? lo : hi, tw2[z]);
      }
    }
   }
  }
  if (!vec) {
    // every load of the tile in flight before the first LDS store
    constexpr int EPT = (2 * P * B * NZ + kFftThreads - 1) / kFftThreads;
    C v[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int f = threadIdx.x + e * kFftThreads;
      if (f < total) {
        const int b = f % nb;
        const int r = f / nb;              // (side, p, z) with z fastest after b
        const int z = r % NZ;
        const int sp = r / NZ;             // side * P + p
        const int side = sp / P, p = sp - side * P;
        v[e] = spec[addr(side, p, b, z)];
      }
    }
    __syncthreads();   // twiddles visible
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int f = threadIdx.x + e * kFftThreads;
      if (f < total) {
        const int b = f % nb;
        const int r = f / nb;
        const int z = r % NZ;
        const int sp = r / NZ;
        buf[Lds<NZ>::at(sp * B + b, z)] = cmul(v[e], tw2[z]);
      }
    }
  }
  __syncthreads();
  // forward z passes over all 2 P B lines (unused tail lines carry stale data and are not stored)
  passes_from<0, 1, NZ, LINES, WidePlan<NZ>>(buf, LINES, tw2, S(-1));

  // contraction: (b, jz) on side 0 with its mirror (b, NZ-1-jz) on side 1
  for (int t = threadIdx.x; t < nb * NZ; t += kFftThreads) {
    const int b = t / NZ;
    const int jz = t - b * NZ;
    const int jx = x0 + b;
    int m;
    S fr;
    table_pos<S>(kappa<S>(jx, nx, dkx), kappa<S>(jy, ny, dky), kappa<S>(jz, NZ, dkz), inv_dkt,
                 m_tab, &m, &fr);
    C X[NV];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const C z = buf[Lds<NZ>::at(p * B + b, jz)];
      const C zb = buf[Lds<NZ>::at((P + p) * B + b, NZ - 1 - jz)];
      X[2 * p] = make_c(S(0.5) * (z.x + zb.x), S(0.5) * (z.y - zb.y));
      if (2 * p + 1 < NV) X[2 * p + 1] = make_c(S(0.5) * (z.y + zb.y), S(-0.5) * (z.x - zb.x));
    }
    C Fk = make_c(S(0), S(0));
    if (WITHF) {
      // F is stored for the first half of the linear k index; the second half is conjugate
      const size_t L = ((size_t)jz * ny + jy) * nx + jx;
      const size_t Lb = N - 1 - L;
      Fk = L < (N + 1) / 2 ? F[L] : cconj(F[Lb]);
    }
    C H[NV];
    contract_point<NV, C, WITHF>(X, Fk, m, fr, chi, qtab, H);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const C a = H[2 * p];
      const C bb = (2 * p + 1 < NV) ? H[2 * p + 1] : make_c(S(0), S(0));
      buf[Lds<NZ>::at(p * B + b, jz)] = make_c(a.x - bb.y, a.y + bb.x);
      buf[Lds<NZ>::at((P + p) * B + b, NZ - 1 - jz)] = make_c(a.x + bb.y, -a.y + bb.x);
    }
  }
  __syncthreads();
  passes_from<0, 1, NZ, LINES, WidePlan<NZ>>(buf, LINES, tw2, S(1));
  if constexpr (kVec) {
   if (vec) {
    for (int f = threadIdx.x; f < 2 * P * H * NZ; f += kFftThreads) {
      const int h = f % H;
      const int r = f / H;
      const int z = r % NZ;
      const int sp = r / NZ;
      const int side = sp / P, p = sp - side * P;
      const C a = cmulc(buf[Lds<NZ>::at(sp * B + 2 * h, z)], tw2[z]);
      const C c = cmulc(buf[Lds<NZ>::at(sp * B + 2 * h + 1, z)], tw2[z]);
      const C lo = side ? c : a, hi = side ? a : c;
      *reinterpret_cast<float4*>(spec + pair_addr(side, p, h, z)) =
          make_float4((float)lo.x, (float)lo.y, (float)hi.x, (float)hi.y);
    }
    return;
   }
  }
  for (int f = threadIdx.x; f < total; f += kFftThreads) {
    const int b = f % nb;
    const int r = f / nb;
    const int z = r % NZ;
    const int sp = r / NZ;
    const int side = sp / P, p = sp - side * P;
    spec[addr(side, p, b, z)] = cmulc(buf[Lds<NZ>::at(sp * B + b, z)], tw2[z]);
  }
}

}  // namespace rism
