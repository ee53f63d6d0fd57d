// Per-solute set-up kernels: solute potential (Eq 22), long-range split
// (Eq 29-30), chi interpolation tables and FFT twiddles.  They run once per
// solve, so they work in FP64 and round only their stored results to FP32.
#pragma once

#include "common.hpp"

namespace rism {

constexpr int kPotThreads = 256;
constexpr int kPotChunk = 256;   // atoms staged in LDS per round

// Solute atoms relative to the grid corner r0 (with the charge in .w), and per
// (atom, site) LJ coefficients beta*4*eps*sigma^12 and beta*4*eps*sigma^6
// (Lorentz-Berthelot mixing).
__global__ void k_prep_atoms(const double* __restrict__ xyz, const double* __restrict__ q,
                             const double* __restrict__ sigma, const double* __restrict__ eps,
                             int n_atoms, double r0x, double r0y, double r0z, double beta,
                             int nv, SiteLJ sites, double4* __restrict__ atoms,
                             double2* __restrict__ lj) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n_atoms) return;
  atoms[a] = make_double4(xyz[3 * a] - r0x, xyz[3 * a + 1] - r0y, xyz[3 * a + 2] - r0z, q[a]);
  for (int g = 0; g < nv; ++g) {
    const double s = 0.5 * (sigma[a] + sites.sigma[g]);
    const double e = sqrt(eps[a] * sites.eps[g]);
    const double s6 = s * s * s * s * s * s;
    lj[(size_t)a * nv + g] = make_double2(beta * 4.0 * e * s6 * s6, beta * 4.0 * e * s6);
  }
}

// w_g = min(beta u_g, cap) - f_g and phi_lr on every grid point.
//   beta u_g = sum_a [beta LJ_ag(dc) + coul_g q_a / dc],  dc = max(d, D_MIN)
//   f_g      = coul_g * phi_lr,  phi_lr = sum_a q_a (1 - e^{-d}) / d
// The uncapped w is accumulated directly as beta LJ + coul_g * phi_sr with
//   phi_sr = sum_a q_a s(d),  s(d) = e^{-d}/d (d >= D_MIN),
//                             s(d) = 1/D_MIN - (1 - e^{-d})/d (d < D_MIN),
// which equals q/dc - q (1 - e^{-d})/d term by term and avoids subtracting two
// long-ranged sums.  Pair terms and sums are FP64 (the twelfth power of a
// rounded FP32 distance would cost ~1e-5 relative in w near the solute).
template <int NV>
__global__ __launch_bounds__(kPotThreads) void k_potential(
    const double4* __restrict__ atoms, const double2* __restrict__ lj, int n_atoms, int nx, int ny,
    int nz, double dr, SiteConsts sc, float* __restrict__ w, float* __restrict__ phi_out) {
  __shared__ double4 s_at[kPotChunk];
  __shared__ double2 s_lj[kPotChunk * NV];
  const size_t N = (size_t)nx * ny * nz;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = idx < N;
  const int ix = (int)(idx % nx);
  const int iy = (int)((idx / nx) % ny);
  const int iz = (int)(idx / ((size_t)nx * ny));
  const double px = ix * dr, py = iy * dr, pz = iz * dr;
  double acc[NV];
#pragma unroll
  for (int g = 0; g < NV; ++g) acc[g] = 0.0;
  double phi_sr = 0.0, phi_lr = 0.0;
  for (int a0 = 0; a0 < n_atoms; a0 += kPotChunk) {
    const int cnt = (n_atoms - a0) < kPotChunk ? (n_atoms - a0) : kPotChunk;
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) s_at[t] = atoms[a0 + t];
    for (int t = threadIdx.x; t < cnt * NV; t += blockDim.x) s_lj[t] = lj[(size_t)a0 * NV + t];
    __syncthreads();
    if (live) {
      for (int a = 0; a < cnt; ++a) {
        const double4 at = s_at[a];
        const double dx = px - at.x, dy = py - at.y, dz = pz - at.z;
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double dc = fmax(d, kDMin);
        const double inv = 1.0 / dc;
        // beyond 38 A, e^{-d} < 2^-54: 1 - e^{-d} rounds to 1 and e^{-d}/d adds
        // below FP64 resolution, so the exponential is skipped there
        const double e = d < 38.0 ? exp(-d) : 0.0;
        // (1 - e^{-d})/d with screening length 1 A; expm1 only where 1 - e^{-d} cancels
        const double lr = (d < 0.5) ? ((d > 1.0e-300) ? -expm1(-d) / d : 1.0) : (1.0 - e) / d;
        const double sr = (d >= kDMin) ? e * inv : 1.0 / kDMin - lr;
        phi_lr += at.w * lr;
        phi_sr += at.w * sr;
        const double s2 = inv * inv;
        const double s6 = s2 * s2 * s2;
#pragma unroll
        for (int g = 0; g < NV; ++g) {
          const double2 c = s_lj[a * NV + g];
          acc[g] += (c.x * s6 - c.y) * s6;
        }
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int g = 0; g < NV; ++g) {
    const double coul = sc.coul64[g];
    const double bu = acc[g] + coul * (phi_sr + phi_lr);
    w[(size_t)g * N + idx] = (float)((bu > kBetaUCap) ? kBetaUCap - coul * phi_lr : acc[g] + coul * phi_sr);
  }
  phi_out[idx] = (float)phi_lr;
}

__device__ inline double kappa_of(int j, int n, double dk) {
  return (2 * j < n) ? (j + 0.5) * dk : (j + 0.5 - n) * dk;
}

// Per-atom, per-axis phase tables exp(-i kappa(j) (R_a - r0)) in FP64.
__global__ void k_phase_tables(const double* __restrict__ xyz, int n_atoms, int nx, int ny, int nz,
                               double r0x, double r0y, double r0z, double dkx, double dky,
                               double dkz, double2* __restrict__ ph) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nsum = nx + ny + nz;
  if (t >= n_atoms * nsum) return;
  const int a = t / nsum;
  int j = t - a * nsum;
  double kap, rel;
  if (j < nx) {
    kap = kappa_of(j, nx, dkx);
    rel = xyz[3 * a] - r0x;
  } else if (j < nx + ny) {
    j -= nx;
    kap = kappa_of(j, ny, dky);
    rel = xyz[3 * a + 1] - r0y;
  } else {
    j -= nx + ny;
    kap = kappa_of(j, nz, dkz);
    rel = xyz[3 * a + 2] - r0z;
  }
  double s, c;
  sincos(kap * rel, &s, &c);
  ph[t] = make_double2(c, -s);
}

// Long-range spectrum of Eq 30 for the first ceil(N/2) k-points in linear order,
// divided by dV (the forward FFT is unnormalised):
//   F(k) = (4 pi beta C / l^2) / (|k|^2 (|k|^2 + l^-2)) / dV * sum_a q_a e^{-i k.(R_a - r0)}
// so that f~_g / dV = q_g F (the 1/N of the inverse sits in the Q table).  The
// other half follows from F(-k) = conj F(k).
__global__ void k_ftilde(const double2* __restrict__ ph, const double4* __restrict__ atoms,
                         int n_atoms, int nx, int ny, int nz, double dkx, double dky, double dkz,
                         double pref, double2* __restrict__ F) {
  const size_t N = (size_t)nx * ny * nz;
  const size_t half = (N + 1) / 2;
  const size_t L = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= half) return;
  const int jx = (int)(L % nx);
  const int jy = (int)((L / nx) % ny);
  const int jz = (int)(L / ((size_t)nx * ny));
  const int nsum = nx + ny + nz;
  double sx = 0.0, sy = 0.0;
  for (int a = 0; a < n_atoms; ++a) {
    const double2* pa = ph + (size_t)a * nsum;
    const double2 e = cmul(cmul(pa[jx], pa[nx + jy]), pa[nx + ny + jz]);
    const double qa = atoms[a].w;
    sx += qa * e.x;
    sy += qa * e.y;
  }
  const double kx = kappa_of(jx, nx, dkx), ky = kappa_of(jy, ny, dky), kz = kappa_of(jz, nz, dkz);
  const double k2 = kx * kx + ky * ky + kz * kz;
  const double s = pref / (k2 * (k2 + 1.0 / (kScreen * kScreen)));
  F[L] = make_double2(s * sx, s * sy);
}

// Interpolation tables with the 1/N of the inverse transform folded in:
//   chi[m][a][b] = chi_ab(m dk) / N,  q[m][b] = sum_a q_a chi_ab(m dk) / N,
// in FP32 (bulk increments) and FP64 (anchor evaluations).
__global__ void k_chi_tables(const double* __restrict__ chi, int nv, int n_k, int m_tab,
                             double inv_n, SiteConsts sc, float* __restrict__ chi32,
                             double* __restrict__ chi64, double* __restrict__ q64) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m_tab * nv) return;
  const int m = t / nv;
  const int b = t - m * nv;
  const int rw32 = chi_row<float>(nv), rw64 = chi_row<double>(nv);
  double qs = 0.0;
  for (int a = 0; a < nv; ++a) {
    const double v = chi[((size_t)a * nv + b) * n_k + m];
    chi32[(size_t)m * rw32 + a * nv + b] = (float)(v * inv_n);
    chi64[(size_t)m * rw64 + a * nv + b] = v * inv_n;
    qs += sc.q64[a] * v;
  }
  if (b == 0) {   // row padding (never read into the arithmetic)
    for (int i = nv * nv; i < rw32; ++i) chi32[(size_t)m * rw32 + i] = 0.0f;
    for (int i = nv * nv; i < rw64; ++i) chi64[(size_t)m * rw64 + i] = 0.0;
  }
  q64[(size_t)m * nv + b] = qs * inv_n;
}

// tw2[m] = exp(-2 pi i m / (2n)), m = 0..2n-1, computed in FP64.
__global__ void k_twiddles(int n, float2* __restrict__ tw32, double2* __restrict__ tw64) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= 2 * n) return;
  double s, c;
  sincospi((double)m / (double)n, &s, &c);
  if (tw32) tw32[m] = make_float2((float)c, (float)(-s));
  if (tw64) tw64[m] = make_double2(c, -s);
}

}  // namespace rism
