// Kernels of the self-consistent iteration (steps 2-7 of "Numerical
// procedure") in the tau-form: tau = t - f, w = min(beta u, cap) - f, so that
//   d = -beta u + t = -w + tau   (Eq 16)
//   c_sr = g - 1 - t + f = g - 1 - tau   (Eq 31)
//   R = t' - t = h + 1 - g   (Eq 33)
// MDIIS is affine invariant (sum c_i = 1), so iterating tau instead of t is
// the same iteration shifted by the constant field f.
//
// Precision.  An FP32 FFT of c_sr has round-off ~1e-7 |c_sr|, and c_sr reaches
// tens to hundreds inside the solute core, which puts a noise floor near the
// rms 1e-6 stopping threshold.  The map is therefore evaluated as a defect
// correction: every few iterations an FP64 "anchor" evaluation computes
// R_ref = R(tau_ref) exactly (double2 transforms); the iterations in between
// transform only the FP32 increment
//   dc = [g(d_ref + delta) - g(d_ref)] - delta,   delta = tau - tau_ref,
// (the analytic long-range term cancels in the difference) and form
//   R = R_ref + dh - dg.
// The increment is small wherever the iteration has converged, so its FP32
// round-off is a small fraction of the current residual.
//
// Storage.  The history slots hold delta = tau - tau_ref, not tau: inside a
// large solute core |tau| reaches 1e3, where the spacing of FP32 values (1e-4)
// would swallow the small updates of a converging iteration.  tau is the
// exact sum tau_ref + delta, formed in FP64 wherever tau itself is needed (the
// anchor evaluation and the outputs).  The reference is a pair of FP32 fields,
// tau_ref + tau_lo (tau_lo the rounding remainder of the FP64 iterate): each
// anchor moves it to the current tau, exactly to about 2^-48, and re-bases
// every stored delta on it.  R_ref is then the exact residual at the very
// reference the FP32 increments are measured from; with tau_ref alone (tau
// rounded to FP32) every FP32 residual would carry the map's response to that
// rounding, up to half an FP32 spacing of tau (~3e-5 where |tau| ~ 1e3).  The
// FP32 kernels read tau_ref only (as d_ref = -w + tau_ref of the closure
// increment, where the remainder is negligible); only FP64 work reads tau_lo.
#pragma once

#include "common.hpp"

namespace rism {

constexpr int kElemThreads = 256;
constexpr int kRedBlocks = 1024;    // fixed block count of the FP64 reductions
constexpr int kRedThreads = 256;

// ---------------------------------------------------------------------------
// State initialisation (a kernel rather than a memset so it can sit in a graph)
// ---------------------------------------------------------------------------
__global__ void k_init_state(IterState* st, float eta, int warm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i < kMaxDepth; ++i) {
    st->stored[i] = 0;
    st->stamp[i] = 0;
    st->coef[i] = 0.0f;
    st->rms_slot[i] = 0.0;
    for (int j = 0; j < kMaxDepth; ++j) st->gram[i][j] = 0.0;
  }
  st->stamp_counter = 0;
  st->dest = 0;
  st->newest = 0;
  st->iter = 0;
  st->done = 0;
  st->converged = 0;
  st->status = RISM3D_OK;
  st->restarts = 0;
  st->final_slot = 0;
  st->eta = eta;
  st->warm = warm;
  st->last_rms = 0.0;
  st->last_rr = 0.0;
  st->ticket = 0;
  st->hold = 0;
}

// Place the starting tau (the caller's, or zero) in history slot 0, where the
// first update reads it; keeps the iteration kernels independent of the call.
// The start: tau_ref = tau0 (or 0) and delta = 0 in the first slot.
__global__ void k_init_tau(const float* __restrict__ tau0, float* __restrict__ slot0,
                           float* __restrict__ tau_ref, float* __restrict__ tau_lo, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    slot0[i] = 0.0f;
    tau_ref[i] = tau0 ? tau0[i] : 0.0f;
    tau_lo[i] = 0.0f;
  }
}

__global__ void k_mark_prepared(IterState* st, unsigned layout_key) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->prepared = kPreparedMagic;
    st->layout_key = layout_key;
    st->done = 1;
    st->final_slot = -1;
  }
}

// ---------------------------------------------------------------------------
// Step 6 + step 2 fused: MDIIS update, in difference form about the newest
// stored pair b (which keeps sum c_i = 1 exact in FP32):
//   tau = tau_b + sum_i c_i (tau_i - tau_b) + eta sum_i c_i R_i,
// stored in the destination slot (as delta = tau - tau_ref); then the closure.  ANCHOR: c_sr = g - 1 - tau
// in FP64 (double2 grid).  Otherwise the FP32 increment dc = dg - delta about
// the anchor, with dg kept for the residual.  Two sites share one complex grid
// (site 2p real part, site 2p+1 imaginary part).
// ---------------------------------------------------------------------------
// V consecutive floats (V = 4: one 16-byte access).
template <int V>
__device__ inline void ldv(const float* __restrict__ p, float* o) {
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) o[i] = p[i];
  }
}
template <int V>
__device__ inline void stv(float* __restrict__ p, const float* v) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) p[i] = v[i];
  }
}

// Per-workgroup copy of what the update needs from the state.
struct UpdateCtl {
  float cf[kMaxDepth];
  float eta;
  int dest, newest, first, M;
};

__device__ inline UpdateCtl load_update_ctl(const IterState* __restrict__ st, int M) {
  UpdateCtl u;
#pragma unroll
  for (int i = 0; i < kMaxDepth; ++i) u.cf[i] = i < M ? st->coef[i] : 0.0f;
  u.eta = st->eta;
  u.dest = st->dest;
  u.newest = st->newest;
  u.first = st->iter == 0 || st->hold != 0;   // the iterate already in slot dest
  u.M = M;
  return u;
}

// The update + closure of V consecutive points n.. of pair p: stores the new tau
// (and dg in the FP32 path) and returns the two sites' FFT inputs.
// ANCHOR: c_sr = g - 1 - tau (FP64).  Otherwise dc = dg - delta.
// The FP32 path takes the closure argument of the reference, d_ref = -w +
// tau_ref + tau_lo, from dref (written by the last anchor) instead of w and
// tau_ref.
template <bool ANCHOR, int V, int MM = kMaxDepth>
__device__ inline void update_points(const UpdateCtl& u, float* __restrict__ tau_hist,
                                     const float* __restrict__ res_hist,
                                     const float* __restrict__ w,
                                     const float* __restrict__ tau_ref,
                                     const float* __restrict__ tau_lo,
                                     const float* __restrict__ dref, float* __restrict__ dg_out,
                                     size_t N, int nv, int p, size_t n, int kind, int order,
                                     double (*o64)[V], float (*o32)[V]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      o64[s][v] = 0.0;
      o32[s][v] = 0.0f;
    }
  for (int s = 0; s < 2; ++s) {
    const int g = 2 * p + s;
    if (g >= nv) break;
    const size_t gn = (size_t)g * N + n;
    float tau[V];   // delta = tau - tau_ref of the new iterate
    if (u.first) {
      ldv<V>(tau_hist + (size_t)u.dest * nv * N + gn, tau);   // the start, placed by k_init_tau
    } else {
      float tb[V], dt[V], dr[V];
      ldv<V>(tau_hist + (size_t)u.newest * nv * N + gn, tb);
#pragma unroll
      for (int v = 0; v < V; ++v) dt[v] = dr[v] = 0.0f;
      // the stored pairs in chunks of K slots: every load of a chunk is in
      // flight before the first is used (the sums keep the slot order)
      constexpr int K = MM <= 5 ? MM : 4;
#pragma unroll
      for (int i0 = 0; i0 < MM; i0 += K) {
        float ti[K][V], ri[K][V];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int i = i0 + k;
          if (i < MM && u.cf[i] != 0.0f) {   // zero beyond M and for unused slots
            ldv<V>(tau_hist + (size_t)i * nv * N + gn, ti[k]);
            ldv<V>(res_hist + (size_t)i * nv * N + gn, ri[k]);
          }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const int i = i0 + k;
          const float c = i < MM ? u.cf[i] : 0.0f;
          if (c != 0.0f) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
              dt[v] += c * (ti[k][v] - tb[v]);
              dr[v] += c * ri[k][v];
            }
          }
        }
      }
#pragma unroll
      for (int v = 0; v < V; ++v) tau[v] = tb[v] + (dt[v] + u.eta * dr[v]);
    }
    stv<V>(tau_hist + (size_t)u.dest * nv * N + gn, tau);
    if (ANCHOR) {
      float wv[V], tr[V], tl[V];
      ldv<V>(w + gn, wv);
      ldv<V>(tau_ref + gn, tr);
      ldv<V>(tau_lo + gn, tl);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double t = ((double)tr[v] + (double)tl[v]) + (double)tau[v];
        o64[s][v] = closure_g(-(double)wv[v] + t, kind, order) - 1.0 - t;
      }
    } else {
      float dr[V], dg[V];
      ldv<V>(dref + gn, dr);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        dg[v] = closure_dg(dr[v], tau[v], kind, order);
        o32[s][v] = dg[v] - tau[v];
      }
      stv<V>(dg_out + gn, dg);
    }
  }
}

template <bool ANCHOR, int V>
__global__ __launch_bounds__(kElemThreads) void k_update_closure(
    const IterState* __restrict__ st, float* __restrict__ tau_hist,
    const float* __restrict__ res_hist, const float* __restrict__ w,
    const float* __restrict__ tau_ref, const float* __restrict__ tau_lo,
    const float* __restrict__ dref, float* __restrict__ dg_out, void* __restrict__ spec, size_t N,
    int nv, int npair, int M, int kind, int order) {
  if (skip_iteration<ANCHOR>(st->done)) return;
  const size_t NQ = N / V;
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)npair * NQ) return;
  const int p = (int)(q / NQ);
  const size_t n = (q - (size_t)p * NQ) * V;
  const UpdateCtl u = load_update_ctl(st, M);
  double o64[2][V];
  float o32[2][V];
  update_points<ANCHOR, V>(u, tau_hist, res_hist, w, tau_ref, tau_lo, dref, dg_out, N, nv, p, n,
                           kind, order, o64, o32);
  const size_t o = (size_t)p * N + n;
  if (ANCHOR) {
    double2* sp = static_cast<double2*>(spec) + o;
#pragma unroll
    for (int v = 0; v < V; ++v) sp[v] = make_double2(o64[0][v], o64[1][v]);
  } else {
    float* sp = reinterpret_cast<float*>(static_cast<float2*>(spec) + o);
    float pk[2 * V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      pk[2 * v] = o32[0][v];
      pk[2 * v + 1] = o32[1][v];
    }
    if constexpr (V == 4) {
      stv<4>(sp, pk);
      stv<4>(sp + 4, pk + 4);
    } else {
      stv<2 * V>(sp, pk);
    }
  }
}

// ---------------------------------------------------------------------------
// Steps 3-4 in k-space: unpack each site pair, c~ = c~sr - f~ (Eq 32), the
// 3D-RISM contraction h~_g = sum_g' c~_g' chi_g'g(|k|) (Eq 13), repack.
// With f~_g = q_g F:  h~_g = sum_g' c~sr_g' chi_g'g - F Q_g,  Q_g = sum_g' q_g' chi_g'g.
// The increments (WITHF = false) carry no long-range term.
// Thread L handles the mirror pair (L, N-1-L): k_(N-1-L) = -k_L.
// ---------------------------------------------------------------------------
// The half-integer k representative of index j on an axis of n points, in the
// precision S of the evaluation (FP64 for the anchors: the interpolation
// weight below is |k| / dk_table ~ 4e2, where an FP32 |k| would leave an
// absolute error ~3e-5 in the weight).
template <typename S>
__device__ inline S kappa(int j, int n, double dk) {
  return (2 * j < n) ? ((S)j + S(0.5)) * (S)dk : ((S)j + S(0.5) - (S)n) * (S)dk;
}

// Table position of |k|: sample m and linear weight fr (Eq 13's chi by linear
// interpolation; beyond the table the last interval's end value).
template <typename S>
__device__ inline void table_pos(S kx, S ky, S kz, double inv_dkt, int m_tab, int* m, S* fr) {
  const S x = sqrt(kx * kx + ky * ky + kz * kz) * (S)inv_dkt;
  if (x >= (S)(m_tab - 1)) {
    *m = m_tab - 2;
    *fr = S(1);
  } else {
    *m = (int)x;
    *fr = x - (S)(*m);
  }
}

// The contraction of Eq 13 at one k-point with the analytic long-range term
// of Eq 32: H_g = sum_g' X_g' chi_g'g(|k|) - F(k) Q_g(|k|), chi and Q linear
// in |k| between table samples m and m+1 (weight fr).  A table row holds the
// NV*NV values of one sample padded to whole 16-byte vectors (chi_row), so a
// row is fetched with NV*NV/4 (FP32) or NV*NV/2 (FP64) vector loads.
__device__ __forceinline__ void unpack_vec(float* d, const float4& v) {
  d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
}
__device__ __forceinline__ void unpack_vec(double* d, const double2& v) {
  d[0] = v.x; d[1] = v.y;
}

template <int NV, typename C, bool WITHF>
__device__ __forceinline__ void contract_point(const C (&X)[NV], C Fk, int m,
                                               typename ScalarOf<C>::type fr,
                                               const typename ScalarOf<C>::type* __restrict__ chi,
                                               const typename ScalarOf<C>::type* __restrict__ qtab,
                                               C (&H)[NV]) {
  using S = typename ScalarOf<C>::type;
  using V = typename std::conditional<sizeof(S) == 4, float4, double2>::type;
  constexpr int RW = chi_row<S>(NV);
  constexpr int VW = (int)(sizeof(V) / sizeof(S));
  S r0[RW], r1[RW];
  const V* v0 = reinterpret_cast<const V*>(chi + (size_t)m * RW);
#pragma unroll
  for (int i = 0; i < RW / VW; ++i) {
    unpack_vec(&r0[i * VW], v0[i]);
    unpack_vec(&r1[i * VW], v0[RW / VW + i]);
  }
#pragma unroll
  for (int g = 0; g < NV; ++g) {
    C acc = make_c(S(0), S(0));
    if (WITHF) {
      const S* q0 = qtab + (size_t)m * NV;
      const S Q = q0[g] + fr * (q0[NV + g] - q0[g]);
      acc = make_c(-Fk.x * Q, -Fk.y * Q);
    }
#pragma unroll
    for (int gp = 0; gp < NV; ++gp) {
      const S c = r0[gp * NV + g] + fr * (r1[gp * NV + g] - r0[gp * NV + g]);
      acc.x += X[gp].x * c;
      acc.y += X[gp].y * c;
    }
    H[g] = acc;
  }
}

template <int NV, typename C, bool WITHF>
__global__ __launch_bounds__(kElemThreads) void k_contract(
    C* __restrict__ spec, int nx, int ny, int nz, double dkx, double dky, double dkz,
    const C* __restrict__ F, const typename ScalarOf<C>::type* __restrict__ chi,
    const typename ScalarOf<C>::type* __restrict__ qtab, double inv_dkt, int m_tab,
    const int* __restrict__ done) {
  using S = typename ScalarOf<C>::type;
  if (done && skip_iteration<std::is_same<C, double2>::value>(*done)) return;
  constexpr int NP = (NV + 1) / 2;
  const size_t N = (size_t)nx * ny * nz;
  const size_t half = (N + 1) / 2;
  const size_t L = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= half) return;
  const size_t Lb = N - 1 - L;
  const int jx = (int)(L % nx);
  const int jy = (int)((L / nx) % ny);
  const int jz = (int)(L / ((size_t)nx * ny));
  int m;
  S fr;
  table_pos<S>(kappa<S>(jx, nx, dkx), kappa<S>(jy, ny, dky), kappa<S>(jz, nz, dkz), inv_dkt,
               m_tab, &m, &fr);
  C X[NV];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const C z = spec[(size_t)p * N + L];
    const C zb = spec[(size_t)p * N + Lb];
    // A = (z + conj zb)/2,  B = (z - conj zb)/(2i)
    X[2 * p] = make_c(S(0.5) * (z.x + zb.x), S(0.5) * (z.y - zb.y));
    if (2 * p + 1 < NV) X[2 * p + 1] = make_c(S(0.5) * (z.y + zb.y), S(-0.5) * (z.x - zb.x));
  }
  C Fk = make_c(S(0), S(0));
  if (WITHF) Fk = F[L];
  C H[NV];
  contract_point<NV, C, WITHF>(X, Fk, m, fr, chi, qtab, H);
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const C a = H[2 * p];
    const C bb = (2 * p + 1 < NV) ? H[2 * p + 1] : make_c(S(0), S(0));
    // W(L) = A + iB;  W(Lb) = conj(A) + i conj(B)
    spec[(size_t)p * N + L] = make_c(a.x - bb.y, a.y + bb.x);
    spec[(size_t)p * N + Lb] = make_c(a.x + bb.y, -a.y + bb.x);
  }
}

// ---------------------------------------------------------------------------
// Step 5 and the MDIIS inner products.  ANCHOR: R = h + 1 - g (Eq 33) in FP64
// from the double2 grid, which also becomes the new anchor (tau_ref, R_ref);
// the stored deltas are re-based on the new tau_ref.
// Otherwise R = R_ref + dh - dg.  R is stored in the destination slot and
// <R, R_i> for every other stored slot and <R, R> are accumulated in FP64;
// per-block partial sums are written in block order (reduced by k_control).
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v, double* lds) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  }
  return s;
}

// The residual of V consecutive points n.. of pair p from the transformed
// values h (hre/him in FP32, h64 in FP64), accumulated into the Gram partials
// acc[0..MM-1] (slots; MM >= the history depth) and acc[MM] (the RMS sum).
template <bool ANCHOR, int V, int MM = kMaxDepth>
__device__ inline void residual_points(const float* hre, const float* him, const double (*h64)[V],
                                       const float* __restrict__ w,
                                       float* __restrict__ tau_hist,
                                       float* __restrict__ res_hist, float* __restrict__ tau_ref,
                                       float* __restrict__ tau_lo, float* __restrict__ r_ref,
                                       float* __restrict__ dref, const float* __restrict__ dg,
                                       size_t N, int nv, int p, size_t n, int dest, unsigned mask,
                                       int kind, int order, const GramW& gw, double* acc) {
  for (int s = 0; s < 2; ++s) {
    const int g = 2 * p + s;
    if (g >= nv) break;
    const double wg = (double)gw.w[g];
    const size_t gn = (size_t)g * N + n;
    const size_t od = (size_t)dest * nv * N + gn;
    float R[V];
    if (ANCHOR) {
      float dl[V], tr[V], tl[V], wv[V], dv[V];
      double shift[V];
      ldv<V>(tau_hist + od, dl);
      ldv<V>(tau_ref + gn, tr);
      ldv<V>(tau_lo + gn, tl);
      ldv<V>(w + gn, wv);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double base = (double)tr[v] + (double)tl[v];   // exact
        const double t = base + (double)dl[v];
        const double gg = closure_g(-(double)wv[v] + t, kind, order);
        R[v] = (float)(h64[s][v] + 1.0 - gg);
        // the new reference hi + lo = t to 2^-48; hi + lo and the shift are exact
        const float hi = (float)t;
        const float lo = (float)(t - (double)hi);
        shift[v] = ((double)hi + (double)lo) - base;
        tr[v] = hi;
        tl[v] = lo;
        dl[v] = (float)((double)dl[v] - shift[v]);
        // the closure argument at the new reference, for the FP32 updates
        dv[v] = (float)(-(double)wv[v] + ((double)hi + (double)lo));
      }
      stv<V>(tau_ref + gn, tr);
      stv<V>(tau_lo + gn, tl);
      stv<V>(dref + gn, dv);
      stv<V>(r_ref + gn, R);
      stv<V>(tau_hist + od, dl);
#pragma unroll
      for (int i = 0; i < kMaxDepth; ++i) {
        if (mask & (1u << i)) {   // every other stored delta moves by the same shift
          float di[V];
          ldv<V>(tau_hist + (size_t)i * nv * N + gn, di);
#pragma unroll
          for (int v = 0; v < V; ++v) di[v] = (float)((double)di[v] - shift[v]);
          stv<V>(tau_hist + (size_t)i * nv * N + gn, di);
        }
      }
    } else {
      float rr[V], dd[V];
      ldv<V>(r_ref + gn, rr);
      ldv<V>(dg + gn, dd);
#pragma unroll
      for (int v = 0; v < V; ++v) R[v] = rr[v] + ((s ? him[v] : hre[v]) - dd[v]);
    }
    stv<V>(res_hist + od, R);
    double rr = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v) rr += (double)R[v] * (double)R[v];
    acc[MM] += rr;                 // unweighted: the RMS
    // the other stored residuals in chunks of K slots, every load of a chunk
    // in flight before the first is used
    constexpr int K = MM <= 5 ? MM : 4;
#pragma unroll
    for (int i0 = 0; i0 < MM; i0 += K) {
      float ri[K][V];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = i0 + k;
        if (i < MM && (mask & (1u << i))) ldv<V>(res_hist + (size_t)i * nv * N + gn, ri[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = i0 + k;
        if (i >= MM) continue;
        if (i == dest) acc[i] += wg * rr;   // weighted Gram diagonal
        if (mask & (1u << i)) {
          double d = 0.0;
#pragma unroll
          for (int v = 0; v < V; ++v) d += (double)R[v] * (double)ri[k][v];
          acc[i] += wg * d;
        }
      }
    }
  }
}

__device__ inline unsigned other_slots(const IterState* __restrict__ st, int M, int dest) {
  unsigned mask = 0;
  for (int i = 0; i < M; ++i)
    if (st->stored[i] && i != dest) mask |= 1u << i;
  return mask;
}

// Write this block's partial sums (fixed block order, reduced in fixed order).
// Partials are column-major: quantity i of workgroup b at i * gridDim.x + b,
// so the control kernel reads each quantity as one contiguous run.  Each
// wavefront reduces every quantity by shuffles (the tree of block_sum); one
// barrier later thread q adds the wavefronts' sums of quantity q in wavefront
// order, as block_sum does.  red holds (MM + 1) * (blockDim.x / 64) doubles.
template <int MM = kMaxDepth>
__device__ inline void write_partials(const double* acc, int M, double* __restrict__ partials,
                                      double* red) {
  const size_t nb = gridDim.x;
  const int nw = (int)(blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= MM; ++i) {
    if (i < M || i == MM) {   // M is uniform: every thread takes the same branches
      double v = acc[i];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if (lane == 0) red[(i < M ? i : M) * nw + wv] = v;
    }
  }
  __syncthreads();
  const int q = (int)threadIdx.x;
  if (q <= M) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[q * nw + i];
    partials[(size_t)q * nb + blockIdx.x] = s;
  }
}

template <bool ANCHOR, int V>
__global__ __launch_bounds__(kRedThreads) void k_residual(
    const IterState* __restrict__ st, const void* __restrict__ spec, const float* __restrict__ w,
    float* __restrict__ tau_hist, float* __restrict__ res_hist, float* __restrict__ tau_ref,
    float* __restrict__ tau_lo, float* __restrict__ r_ref, float* __restrict__ dref,
    const float* __restrict__ dg, size_t N, int nv, int npair, int M, int kind, int order,
    double* __restrict__ partials, GramW gw) {
  if (skip_iteration<ANCHOR>(st->done)) return;
  __shared__ double red[(kMaxDepth + 1) * (kRedThreads / 64)];
  const int dest = st->dest;
  const unsigned mask = other_slots(st, M, dest);
  double acc[kMaxDepth + 1];
#pragma unroll
  for (int i = 0; i <= kMaxDepth; ++i) acc[i] = 0.0;
  const size_t NQ = N / V;
  const size_t total = (size_t)npair * NQ;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(q / NQ);
    const size_t n = (q - (size_t)p * NQ) * V;
    const size_t o = (size_t)p * N + n;
    float hre[V], him[V];
    double h64[2][V];
    if (ANCHOR) {
      const double2* sp = static_cast<const double2*>(spec) + o;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double2 t = sp[v];
        h64[0][v] = t.x;
        h64[1][v] = t.y;
      }
    } else {
      const float* sp = reinterpret_cast<const float*>(static_cast<const float2*>(spec) + o);
      float pk[2 * V];
      if constexpr (V == 4) {
        ldv<4>(sp, pk);
        ldv<4>(sp + 4, pk + 4);
      } else {
        ldv<2 * V>(sp, pk);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        hre[v] = pk[2 * v];
        him[v] = pk[2 * v + 1];
      }
    }
    residual_points<ANCHOR, V>(hre, him, h64, w, tau_hist, res_hist, tau_ref, tau_lo, r_ref, dref,
                               dg,
                               N, nv, p, n, dest, mask, kind, order, gw, acc);
  }
  write_partials(acc, M, partials, red);
}

// One control step on a (shared-memory) copy of the state; single thread.
// theta of Eq 36 from the stored weighted Gram entries of the newest (0) and
// the two previous (1, 2) residuals; false when the 2x2 system is singular.
__device__ inline bool anderson_theta(const IterState& st, int s0, int s1, int s2, double* theta) {
  const double g00 = st.gram[s0][s0], g01 = st.gram[s0][s1], g02 = st.gram[s0][s2];
  const double g11 = st.gram[s1][s1], g12 = st.gram[s1][s2], g22 = st.gram[s2][s2];
  const double a11 = g00 - 2.0 * g01 + g11;   // (D1, D1), D_i = R0 - R_i
  const double a12 = g00 - g01 - g02 + g12;   // (D1, D2)
  const double a22 = g00 - 2.0 * g02 + g22;   // (D2, D2)
  const double r1 = g00 - g01, r2 = g00 - g02;  // (R0, D_i)
  const double det = a11 * a22 - a12 * a12;
  if (!(fabs(det) > 1e-12 * fmax(a11 * a22, 1e-300))) return false;
  theta[0] = (r1 * a22 - r2 * a12) / det;
  theta[1] = (a11 * r2 - a12 * r1) / det;
  return true;
}

// accel: RISM3D_MDIIS or RISM3D_ANDERSON (shifts as1, as2; mixing eta_static).
// The control workgroup: 1024 threads, so the thousands of per-workgroup
// partial rows of the residual kernels are summed in a few rounds.
constexpr int kCtlThreads = 1024;

struct ControlScratch {
  IterState st;
  double wsum[kCtlThreads / 64][kMaxDepth + 1];
  double sums[kMaxDepth + 1];
  double c[kMaxDepth];
  double rms;
  int slot[kMaxDepth];
  int m;                        // stored pairs
  int mode;                     // what the rest of the step does (kCtl*)
};

constexpr int kCtlDone = 0;      // the step ended (finished, verify, or max_iter)
constexpr int kCtlSolve = 1;     // MDIIS with m > 1: bordered solve, then coefficients
constexpr int kCtlDirect = 2;    // Anderson, or MDIIS with one pair: coefficients directly

// Lane `lane` (uniform) of a double held by every lane of the wavefront.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders the shared-memory accesses of the lanes of one wavefront (the lanes
// run in lockstep; the fences keep the compiler from moving accesses across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One control step (steps 6-7, Eq 40-41; Eq 34-39 for modified Anderson) on
// the state held in shared memory, by the 64 lanes of the first wavefront of
// the control workgroup (only they call it): lane 0 does the bookkeeping,
// the lanes order the stored slots and solve the bordered MDIIS system.  anchor: the evaluation just
// finished was the exact FP64 one.  The stopping test of Eq 41 is decided on
// exact residuals only: an FP32 residual (R_ref + dh - dg, an estimate) below
// tol holds its iterate in slot dest and asks for the next FP64 evaluation
// to re-evaluate it (kDoneVerify); that evaluation either finishes the solve
// or continues it as an ordinary step whose residual is exact.
//
// MDIIS (Eq 40, with the history policy of the design notes): minimise
// |sum c_i R_i|^2 subject to sum c_i = 1 over the stored pairs, oldest
// first: the bordered system [[B, -1], [-1^T, 0]] [c; lambda] = [0; -1] with
// B_ij = <R_i, R_j> / max_i B_ii, Gaussian elimination with partial
// pivoting (first row of largest magnitude) in FP64.  A pivot below 1e-12
// restarts from the stored pair of smallest RMS, and so does a new RMS above
// 10x the smallest stored one (the new pair is then dropped).
template <int MM>
__device__ void control_step(ControlScratch& cs, const double* sums, int M, double inv_count,
                             double tol, int max_iter, float eta_static, int eta_dynamic,
                             int accel, double as1, double as2, int anchor) {
  IterState& st = cs.st;
  const int t = threadIdx.x;
  const bool anderson = accel == RISM3D_ANDERSON;
  if (t == 0) {
    const int dest = st.dest;
    const double rr = sums[M];
    const double rms = sqrt(rr * inv_count);
    cs.rms = rms;
    cs.mode = kCtlDone;
    st.hold = 0;
    st.done = 0;
    st.iter += 1;
    st.last_rms = rms;
    st.last_rr = rr;
    if (!(rr == rr) || rr > 1.0e300) {
      st.status = RISM3D_E_NONFINITE;
      st.final_slot = dest;
      st.done = kDoneFinished;
    } else if (rms < tol) {
      st.final_slot = dest;
      if (anchor) {
        st.converged = 1;
        st.done = kDoneFinished;
      } else {
        st.stored[dest] = 0;   // its old pair was overwritten; the FP64 pass stores it anew
        st.hold = 1;
        st.done = kDoneVerify;
      }
    } else if (st.iter >= max_iter) {
      st.status = RISM3D_E_NOCONV;
      st.final_slot = dest;
      st.done = kDoneFinished;
    } else {
      // The destination slot's old pair (the oldest, when the ring was full)
      // has been overwritten by the new iterate: drop it.
      st.stored[dest] = 0;
      int best = -1;
      double best_rms = 0.0;
      for (int i = 0; i < M; ++i) {
        if (st.stored[i] && (best < 0 || st.rms_slot[i] < best_rms)) {
          best = i;
          best_rms = st.rms_slot[i];
        }
      }
      if (!anderson && best >= 0 && rms > 10.0 * best_rms) {
        for (int i = 0; i < M; ++i) st.stored[i] = (i == best);
        st.newest = best;
        st.restarts += 1;
      } else {
        st.stored[dest] = 1;
        st.newest = dest;
        st.rms_slot[dest] = rms;
        st.stamp[dest] = ++st.stamp_counter;
        for (int i = 0; i < M; ++i) {
          if (st.stored[i] && i != dest) {
            st.gram[dest][i] = sums[i];
            st.gram[i][dest] = sums[i];
          }
        }
        st.gram[dest][dest] = anderson ? sums[dest] : rr;   // weighted for Anderson (Eq 38)
      }
      int m = 0;
      for (int i = 0; i < M; ++i) m += st.stored[i] != 0;
      cs.m = m;
      cs.mode = (!anderson && m > 1) ? kCtlSolve : kCtlDirect;
    }
  }
  wave_sync();
  if (cs.mode == kCtlDone) return;
  const int m = cs.m;
  // stored slots, oldest first: a slot's rank is the number of older ones
  if (t < M && st.stored[t]) {
    int r = 0;
    for (int j = 0; j < M; ++j) r += st.stored[j] && st.stamp[j] < st.stamp[t];
    cs.slot[r] = t;
  }
  wave_sync();
  bool solved = true;
  if (cs.mode == kCtlSolve) {
    // The bordered system in registers: lane j holds column j (lane n the
    // right-hand side); pivots, the pivot column and the solution reach the
    // other lanes by readlane.  The operations and their order are those of
    // Gaussian elimination with partial pivoting on the whole array.
    constexpr int NM = MM + 1;
    const int n = m + 1;
    double scale = 0.0;
    for (int i = 0; i < m; ++i) scale = fmax(scale, st.gram[cs.slot[i]][cs.slot[i]]);
    double a[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) {
      double v = 0.0;
      if (i < n && t <= n) {
        if (t == n) v = i == m ? -1.0 : 0.0;                 // right-hand side
        else if (i < m && t < m) v = st.gram[cs.slot[i]][cs.slot[t]] / scale;
        else if (i == m && t == m) v = 0.0;
        else v = -1.0;                                      // the border
      }
      a[i] = v;
    }
    double min_piv = 1.0e300;
#pragma unroll
    for (int col = 0; col < NM; ++col) {
      if (col < n && solved) {
        // partial pivoting: the first row of largest magnitude in column col
        int pl = col;
        double bl = fabs(a[col]);
#pragma unroll
        for (int r = col + 1; r < NM; ++r)
          if (r < n && fabs(a[r]) > bl) {
            bl = fabs(a[r]);
            pl = r;
          }
        const int piv = __builtin_amdgcn_readlane(pl, col);
        min_piv = fmin(min_piv, readlane_d(bl, col));
        if (piv != col) {
          double ap = a[col];
#pragma unroll
          for (int r = col + 1; r < NM; ++r)
            if (r == piv) ap = a[r];
#pragma unroll
          for (int r = col + 1; r < NM; ++r)
            if (r == piv) a[r] = a[col];
          a[col] = ap;
        }
        const double pv = readlane_d(a[col], col);
        if (!(fabs(pv) >= 1.0e-300)) {
          solved = false;   // uniform: every lane reads the same pivot
        } else {
          double f[NM];
#pragma unroll
          for (int r = col + 1; r < NM; ++r) f[r] = readlane_d(a[r], col) / pv;
          const bool upd = t >= col && t <= n;
#pragma unroll
          for (int r = col + 1; r < NM; ++r)
            if (r < n && upd) a[r] -= f[r] * a[col];
        }
      }
    }
    if (solved && min_piv < 1.0e-12) solved = false;
    if (solved) {
      // back substitution, column by column: x_r = b_r / A_rr, then every
      // row above drops its A_ir x_r
#pragma unroll
      for (int r = NM - 1; r >= 0; --r) {
        if (r < n) {
          const double xr = readlane_d(a[r], n) / readlane_d(a[r], r);
          if (t == n) a[r] = xr;
#pragma unroll
          for (int i = 0; i < r; ++i) {
            const double air = readlane_d(a[i], r);
            if (t == n) a[i] -= air * xr;
          }
        }
      }
      if (t == n) {
#pragma unroll
        for (int i = 0; i < NM - 1; ++i)
          if (i < m) cs.c[i] = a[i];
      }
    }
    wave_sync();
  }
  if (t == 0) {
    int* slot = cs.slot;
    double* c = cs.c;
    int mm = m;
    if (anderson) {
      // Picard for the first two steps (and for a singular theta system), then
      // X = sum c_k (X_k + b R_k) with c = (theta_2 + s_2, theta_1 + s_1,
      // 1 - sum(theta + s)) on the three pairs oldest first (Eq 34-39)
      double theta[2];
      for (int i = 0; i < mm; ++i) c[i] = 0.0;
      c[mm - 1] = 1.0;
      if (mm == 3 && anderson_theta(st, slot[2], slot[1], slot[0], theta)) {
        const double k1 = theta[0] + as1, k2 = theta[1] + as2;
        c[2] = 1.0 - k1 - k2;
        c[1] = k1;
        c[0] = k2;
      }
    } else if (mm == 1) {
      c[0] = 1.0;
    } else if (!solved) {
      // ill-conditioned subspace: restart from the best stored pair
      int b = slot[0];
      for (int i = 1; i < mm; ++i)
        if (st.rms_slot[slot[i]] < st.rms_slot[b]) b = slot[i];
      for (int i = 0; i < M; ++i) st.stored[i] = (i == b);
      st.newest = b;
      slot[0] = b;
      mm = 1;
      c[0] = 1.0;
      st.restarts += 1;
    }
    for (int i = 0; i < M; ++i) st.coef[i] = 0.0f;
    for (int i = 0; i < mm; ++i) st.coef[slot[i]] = (float)c[i];
    float eta = eta_static;
    if (eta_dynamic && !anderson) eta = (float)fmin(fmax(-0.2 * log(cs.rms), 0.1), 1.0);
    st.eta = eta;
    // Next destination: a free slot while the ring is not full, else the oldest.
    int next = -1;
    if (mm < M) {
      for (int i = 0; i < M; ++i)
        if (!st.stored[i]) {
          next = i;
          break;
        }
    } else {
      next = slot[0];
    }
    st.dest = next;
  }
}

// Shared-memory scratch of the control step.
// Reduce the partials of `nblocks` blocks in fixed order and run one control
// step on the state (anchor: the evaluation was the FP64 one); all threads of
// the calling workgroup participate.
// MM bounds the history depth (M <= MM): each thread holds MM + 1 sums.
template <int MM = kMaxDepth>
__device__ __forceinline__ void control_block(IterState* __restrict__ st_g,
                                     const double* __restrict__ partials, int nblocks, int M,
                                     double inv_count, double tol, int max_iter, float eta_static,
                                     int eta_dynamic, int accel, double as1, double as2,
                                     int anchor, double2* __restrict__ hist, ControlScratch& cs) {
  {
    const int* src = reinterpret_cast<const int*>(st_g);
    int* dst = reinterpret_cast<int*>(&cs.st);
    for (int i = threadIdx.x; i < (int)(sizeof(IterState) / sizeof(int)); i += blockDim.x)
      dst[i] = src[i];
  }
  // Each thread sums its strided workgroups b = t, t + T, ... for every
  // quantity (quantity q is the contiguous run partials[q * nblocks + b]).
  // The loads of U workgroups and all quantities are issued before any
  // addition and without branches (quantities past M re-read quantity M,
  // workgroups past the end re-read the last one; both add zero), so the
  // round trip to rows just written by other CUs is paid once per U
  // workgroups.  Then one LDS pass combines the per-wave sums in fixed order.
  constexpr int U = MM <= 5 ? 6 : 2;
  double v[MM + 1];
#pragma unroll
  for (int q = 0; q <= MM; ++q) v[q] = 0.0;
  const int T = (int)blockDim.x;
  for (int b = threadIdx.x; b < nblocks; b += U * T) {
    double r[U][MM + 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int bb = b + u * T;
      const size_t bc = (size_t)(bb < nblocks ? bb : nblocks - 1);
#pragma unroll
      for (int q = 0; q <= MM; ++q)
        r[u][q] = partials[(size_t)(q <= M ? q : M) * (size_t)nblocks + bc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = b + u * T < nblocks;
#pragma unroll
      for (int q = 0; q <= MM; ++q) v[q] += (in && q <= M) ? r[u][q] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q <= MM; ++q) {
    if (q <= M) {
      for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
      if ((threadIdx.x & 63) == 0) cs.wsum[threadIdx.x >> 6][q] = v[q];
    }
  }
  __syncthreads();
  if (threadIdx.x <= M) {
    double t = 0.0;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) t += cs.wsum[wv][threadIdx.x];
    cs.sums[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x < 64)
    control_step<MM>(cs, cs.sums, M, inv_count, tol, max_iter, eta_static, eta_dynamic, accel, as1,
                 as2, anchor);
  __syncthreads();
  if (threadIdx.x == 0) {
    // residual history: the RMS of evaluation i (1-based) and whether it was exact
    const int it = cs.st.iter;
    if (it >= 1 && it <= kHistLen) hist[it - 1] = make_double2(cs.st.last_rms, anchor ? 1.0 : 0.0);
  }
  {
    const int* src = reinterpret_cast<const int*>(&cs.st);
    int* dst = reinterpret_cast<int*>(st_g);
    for (int i = threadIdx.x; i < (int)(sizeof(IterState) / sizeof(int)); i += blockDim.x)
      dst[i] = src[i];
  }
}

template <int MM = kMaxDepth>
__global__ __launch_bounds__(kCtlThreads) void k_control(
    IterState* __restrict__ st_g, const double* __restrict__ partials, int nblocks, int M,
    double inv_count, double tol, int max_iter, float eta_static, int eta_dynamic,
    int accel, double as1, double as2, int anchor, double2* __restrict__ hist, size_t bstride) {
  __shared__ ControlScratch cs;
  st_g = member_ptr(st_g, bstride);
  if (anchor ? skip_iteration<true>(st_g->done) : skip_iteration<false>(st_g->done)) return;
  partials = member_ptr(partials, bstride);
  hist = member_ptr(hist, bstride);
  control_block<MM>(st_g, partials, nblocks, M, inv_count, tol, max_iter, eta_static, eta_dynamic,
                accel, as1, as2, anchor, hist, cs);
}

// ---------------------------------------------------------------------------
// Outputs: g of the accepted iterate, and tau itself.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kElemThreads) void k_output(
    const IterState* __restrict__ st, const float* __restrict__ tau_hist,
    const float* __restrict__ tau_ref, const float* __restrict__ tau_lo,
    const float* __restrict__ w, size_t N, int nv, int kind, int order,
    float* __restrict__ g_out, float* __restrict__ tau_out) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nv * N) return;
  const int slot = st->final_slot;
  if (slot < 0) return;
  const double tau = ((double)tau_ref[idx] + (double)tau_lo[idx]) +
                     (double)tau_hist[(size_t)slot * nv * N + idx];
  if (g_out) g_out[idx] = (float)closure_g(-(double)w[idx] + tau, kind, order);
  if (tau_out) tau_out[idx] = (float)tau;
}

// ---------------------------------------------------------------------------
// Eq 17 / 18 / PSE-n free-energy density, summed per site in FP64.
//   h = g - 1,  c = g - 1 - t = g - 1 - tau - f,  d = -w + tau
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRedThreads) void k_sfe_partial(
    const IterState* __restrict__ st, const float* __restrict__ tau_hist,
    const float* __restrict__ tau_ref, const float* __restrict__ tau_lo,
    const float* __restrict__ w, const float* __restrict__ phi_lr, size_t N, int nv, int kind,
    int order, SiteConsts sc, double* __restrict__ partials) {
  // partials[block][2 nv]: the free-energy density sums, then the sums of c
  __shared__ double red[kRedThreads / 64];
  const int slot = st->final_slot;
  if (slot < 0) return;
  double inv_fact = 1.0;
  for (int i = 2; i <= order + 1; ++i) inv_fact /= (double)i;
  for (int g = 0; g < nv; ++g) {
    double acc = 0.0, acc_c = 0.0;
    const float* tau = tau_hist + ((size_t)slot * nv + g) * N;
    const float* tr = tau_ref + (size_t)g * N;
    const float* tl = tau_lo + (size_t)g * N;
    const float* wg = w + (size_t)g * N;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
      const double t = ((double)tr[n] + (double)tl[n]) + (double)tau[n];
      const double d = -(double)wg[n] + t;
      const double gg = closure_g(d, kind, order);
      const double h = gg - 1.0;
      const double c = h - t - (double)sc.coul[g] * (double)phi_lr[n];
      double phi = -c - 0.5 * h * c;
      if (kind == RISM3D_HNC) phi += 0.5 * h * h;
      else if (kind == RISM3D_KH) phi += (h < 0.0) ? 0.5 * h * h : 0.0;
      else phi += 0.5 * h * h - ((h > 0.0) ? pow(d, (double)(order + 1)) * inv_fact : 0.0);
      acc += phi;
      acc_c += c;
    }
    const double s = block_sum(acc, red);
    const double sc_sum = block_sum(acc_c, red);
    if (threadIdx.x == 0) {
      partials[(size_t)blockIdx.x * 2 * nv + g] = s;
      partials[(size_t)blockIdx.x * 2 * nv + nv + g] = sc_sum;
    }
  }
}

// out[g] = k_B T rho_g dV sum Phi_g (Eq 17/18), out[kMaxSites] their total,
// out[kMaxSites + 1 + g] = rho_g dV sum c_g (the integral of Eq 19).
__global__ __launch_bounds__(kRedThreads) void k_sfe_reduce(const double* __restrict__ partials,
                                                            int nblocks, int nv, double scale,
                                                            double dv, SiteConsts sc,
                                                            double* __restrict__ out) {
  __shared__ double red[kRedThreads / 64];
  double total = 0.0;
  for (int g = 0; g < nv; ++g) {
    double v = 0.0, vc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      v += partials[(size_t)b * 2 * nv + g];
      vc += partials[(size_t)b * 2 * nv + nv + g];
    }
    const double s = block_sum(v, red);
    const double s_c = block_sum(vc, red);
    if (threadIdx.x == 0) {
      out[g] = s * sc.rho[g] * scale;
      out[kMaxSites + 1 + g] = s_c * sc.rho[g] * dv;
      total += out[g];
    }
  }
  if (threadIdx.x == 0) out[kMaxSites] = total;
}

// Copy of one history slot (the residual of a single map evaluation).
__global__ void k_copy_floats(const float* __restrict__ src, float* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// The history slot of the accepted iterate (final_slot) of n = nv N floats.
__global__ void k_copy_final_slot(const IterState* __restrict__ st,
                                  const float* __restrict__ hist, float* __restrict__ dst,
                                  size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = st->final_slot;
  if (i < n && slot >= 0) dst[i] = hist[(size_t)slot * n + i];
}

// The next evaluation re-evaluates the iterate of a solved workspace (the
// accepted slot, reference + increment, without rounding).
__global__ void k_hold_final(IterState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->dest = st->final_slot;
  st->hold = 1;
  st->done = 0;
  st->status = RISM3D_OK;
}

// The next evaluation takes delta[n] (n = nv N) as its increment over the
// reference: written into slot dest, which the update then leaves as it is.
__global__ void k_set_increment(IterState* st, float* __restrict__ tau_hist,
                                const float* __restrict__ delta, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int slot = st->dest;
  if (i < n) tau_hist[(size_t)slot * n + i] = delta[i];
  if (i == 0) {
    st->hold = 1;
    st->final_slot = slot;
  }
}

}  // namespace rism
