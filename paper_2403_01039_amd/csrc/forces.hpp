// Gradient of the solvation free energy with respect to the solute atom
// positions: the solvent term of the derivative of the MM/3D-RISM free energy
// (section "Hybrid implementation", the derivative of Eq 23),
//
//   d(dmu)/dR_a = sum_g rho_g \int g_g(r) d u_g(r) / dR_a dr,
//
// with u_g the solute-solvent potential of Eq 22.  On the grid the integral is
// the box sum dV sum_n.  Per pair, with d = |r - R_a| and the beta-scaled
// coefficients of k_prep_atoms (A = beta 4 eps sigma^12, B = beta 4 eps
// sigma^6, coul_g = beta C q_g):
//
//   d(beta u_ag)/dR_a = S (R_a - r),   S = -coul_g q_a / d^3 - 12 A / d^14 + 6 B / d^8.
//
// Below d = D_MIN the potential is the clamped constant, so such pairs add
// nothing.  Pair terms and sums are FP64; g is the float32 field the solve
// returns.
//
// Work split: a workgroup holds 64 atoms (one per lane; its four waves take the
// same atoms) and walks tiles of 256 grid points.  A tile's per-point data
// (coordinates, rho_g g_g, and the atom-independent Coulomb weight
// sum_g rho_g g_g coul_g) sit in LDS and are read as broadcasts; points where
// every g_g is 0 (inside the solute core) are skipped by whole waves.  Each
// workgroup leaves one FP64 partial per (atom, component); a second kernel adds
// them in a fixed order, so the result does not depend on scheduling.
#pragma once

#include "common.hpp"

namespace rism {

constexpr int kGradThreads = 256;       // four waves
constexpr int kGradAtoms = 64;          // atoms per workgroup (one per lane)
constexpr int kGradTile = 256;          // grid points staged per round
constexpr double kGradDMin2 = 1.0e-4;   // D_MIN^2 (D_MIN = 0.01 A)

template <int NV>
__global__ __launch_bounds__(kGradThreads) void k_sfe_grad(
    const double4* __restrict__ atoms, const double2* __restrict__ lj, int n_atoms,
    const float* __restrict__ g, int nx, int ny, size_t N, double dr, SiteConsts sc,
    double* __restrict__ out, double scale) {
  __shared__ double s_xyz[3][kGradTile];
  __shared__ double s_rg[NV][kGradTile];
  __shared__ double s_gc[kGradTile];
  __shared__ int s_live[kGradTile];
  __shared__ double s_red[kGradThreads / 64][kGradAtoms][3];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int atom = blockIdx.y * kGradAtoms + lane;
  const int a_ld = atom < n_atoms ? atom : n_atoms - 1;   // idle lanes repeat the last atom
  const double4 at = atoms[a_ld];
  double a12[NV], b6[NV];
#pragma unroll
  for (int s = 0; s < NV; ++s) {
    const double2 c = lj[(size_t)a_ld * NV + s];
    a12[s] = 12.0 * c.x;
    b6[s] = 6.0 * c.y;
  }
  double gx = 0.0, gy = 0.0, gz = 0.0;

  const size_t tiles = (N + kGradTile - 1) / kGradTile;
  for (size_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const size_t p0 = tile * kGradTile;
    const int cnt = (int)((N - p0) < (size_t)kGradTile ? (N - p0) : (size_t)kGradTile);
    __syncthreads();   // the previous tile's LDS is no longer read
    for (int t = threadIdx.x; t < cnt; t += kGradThreads) {
      const size_t p = p0 + t;
      const int ix = (int)(p % nx);
      const int iy = (int)((p / nx) % ny);
      const int iz = (int)(p / ((size_t)nx * ny));
      s_xyz[0][t] = ix * dr;
      s_xyz[1][t] = iy * dr;
      s_xyz[2][t] = iz * dr;
      double gc = 0.0;
      int live = 0;
#pragma unroll
      for (int s = 0; s < NV; ++s) {
        const float gv = g[(size_t)s * N + p];
        live |= gv != 0.0f;
        const double rg = sc.rho[s] * (double)gv;
        s_rg[s][t] = rg;
        gc += rg * sc.coul64[s];
      }
      s_gc[t] = gc;
      s_live[t] = live;
    }
    __syncthreads();
    for (int t = wave; t < cnt; t += kGradThreads / 64) {
      if (!s_live[t]) continue;   // the same point for every lane of the wave
      const double dx = s_xyz[0][t] - at.x, dy = s_xyz[1][t] - at.y, dz = s_xyz[2][t] - at.z;
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < kGradDMin2) continue;
      const double inv = 1.0 / sqrt(d2);
      const double inv2 = inv * inv;
      const double inv6 = inv2 * inv2 * inv2;
      double sa = 0.0, sb = 0.0;
#pragma unroll
      for (int s = 0; s < NV; ++s) {
        const double rg = s_rg[s][t];
        sa += a12[s] * rg;
        sb += b6[s] * rg;
      }
      // S summed over sites with the weights rho_g g_g; the gradient adds S (R - r)
      const double S = -at.w * s_gc[t] * inv2 * inv - inv6 * inv2 * (inv6 * sa - sb);
      gx -= S * dx;
      gy -= S * dy;
      gz -= S * dz;
    }
  }

  s_red[wave][lane][0] = gx;
  s_red[wave][lane][1] = gy;
  s_red[wave][lane][2] = gz;
  __syncthreads();
  if (wave == 0 && atom < n_atoms) {
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v = s_red[0][lane][c];
#pragma unroll
      for (int w = 1; w < kGradThreads / 64; ++w) v += s_red[w][lane][c];
      r[c] = v * scale;
    }
    double* o = out + ((size_t)blockIdx.x * n_atoms + atom) * 3;
    o[0] = r[0];
    o[1] = r[1];
    o[2] = r[2];
  }
}

// out[i] = sum over the nb partial rows of part[b][i], in row order.
__global__ void k_sfe_grad_reduce(const double* __restrict__ part, int nb, int n3,
                                  double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double v = 0.0;
  for (int b = 0; b < nb; ++b) v += part[(size_t)b * n3 + i];
  out[i] = v;
}

}  // namespace rism
