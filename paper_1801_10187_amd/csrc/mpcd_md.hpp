// Molecular dynamics of solute bead chains between MPCD collisions (the MD
// side of the solute coupling), kept apart from the MPCD kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpcd {

// ------------------------------------------------ MD for bead chains
// Velocity Verlet (sec. 3.6, sec. 4.3: solutes move by MD between
// collisions) for chains of `len` beads with harmonic bonds
// U = k/2 (|r_{i+1} - r_i| - b)^2, minimum image in the periodic box. One
// block per chain, one thread per bead; the chain's positions wait in LDS
// for the force evaluation of each substep. Positions are wrapped into
// [0, L) after each drift (x mod L, then a result that rounds to L is 0).
// A drift leaves y = x + dt v in (-L, 2L) but for huge velocities: there
// fmod(y, L) is y, or y - L (exact: L <= y < 2L), taken without the
// library's general remainder.
// Forces on bead i: the bond to i - 1 first, then the bond to i + 1.
// Minimum image d - L rint(d / L). For |d| < L (two positions in [0, L))
// the rounded quotient is 1 exactly when d > L/2 (a quotient that rounds to
// 0.5 has d <= L/2, and a tie rounds to even, 0), -1 when d < -L/2, and a
// zero carrying the sign of d otherwise; the general form is kept for other d.
__device__ inline double min_image(double d, double L) {
  double n;
  if (fabs(d) < L) {
    const double h = 0.5 * L;
    n = d > h ? 1.0 : (d < -h ? -1.0 : copysign(0.0, d));
  } else {
    n = rint(d / L);
  }
  return d - L * n;
}

__device__ inline void bond_pair(const double* pi, const double* pj, const double L[3], double k,
                                 double b, double f[3]) {
  double d[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) d[c] = min_image(pj[c] - pi[c], L[c]);
  const double r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  const double fm = ((-k) * (r - b)) / r;
#pragma unroll
  for (int c = 0; c < 3; ++c) f[c] = fm * d[c];  // on j
}

__global__ __launch_bounds__(1024) void k_md_chains(double* __restrict__ pos, double* __restrict__ vel,
                                                    const double* __restrict__ mass, uint32_t len,
                                                    double L0, double L1, double L2, double k, double b,
                                                    double dt, int nsteps) {
  extern __shared__ double s_p[];  // [len][3]
  const uint32_t i = threadIdx.x;
  const bool on = i < len;
  const size_t row = ((size_t)blockIdx.x * len + i) * 3;
  const double L[3] = {L0, L1, L2};
  double p[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0}, m = 1.0;
  if (on) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p[c] = pos[row + c];
      v[c] = vel[row + c];
      s_p[3 * i + c] = p[c];
    }
    m = mass[(size_t)blockIdx.x * len + i];
  }
  __syncthreads();
  auto force = [&](double f[3]) {
    f[0] = f[1] = f[2] = 0.0;
    if (!on) return;
    double g[3];
    if (i > 0) {
      bond_pair(&s_p[3 * (i - 1)], &s_p[3 * i], L, k, b, g);
#pragma unroll
      for (int c = 0; c < 3; ++c) f[c] = f[c] + g[c];
    }
    if (i + 1 < len) {
      bond_pair(&s_p[3 * i], &s_p[3 * (i + 1)], L, k, b, g);
#pragma unroll
      for (int c = 0; c < 3; ++c) f[c] = f[c] + (-g[c]);
    }
  };
  double f[3];
  force(f);
  const double h = 0.5 * dt;
  for (int s = 0; s < nsteps; ++s) {
    __syncthreads();  // every force read the old positions
    if (on) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[c] = v[c] + (h * f[c]) / m;
        const double y = p[c] + dt * v[c];
        double x = (y > -L[c] && y < 2.0 * L[c]) ? (y >= L[c] ? y - L[c] : y) : fmod(y, L[c]);
        if (x < 0.0) x = x + L[c];
        if (x >= L[c]) x = 0.0;
        p[c] = x + 0.0;  // -0 -> +0
        s_p[3 * i + c] = p[c];
      }
    }
    __syncthreads();
    force(f);
    if (on) {
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = v[c] + (h * f[c]) / m;
    }
  }
  if (on) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pos[row + c] = p[c];
      vel[row + c] = v[c];
    }
  }
}

}  // namespace mpcd
