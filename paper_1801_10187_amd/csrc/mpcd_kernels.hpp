// Kernels of the SRD step on gfx950 (wave64, 160 KB LDS per CU, 8 XCDs).
//
// Data layout in HBM (structure of arrays, one array per component so every
// per-particle access is a unit-stride stream):
//   FP64 form: x[3][N], v[3][N] double.
//   FP32 form: h[N] home cell packed 10:10:10, o[3][N] float offset in the
//              home cell, v[3][N] float.
//   tag[N] uint32 (particle identity), all of the above double-buffered.
//   cr[N] (cell, rank) of each particle in the current order, perm[N] the
//   cell-ordered list, count[C] / off[C+1] per-cell occupancy and offsets.
//
// One step in steady state is: scan(count) -> list(perm) -> collide. The
// collide kernel reads each cell's particles through perm, reduces them per
// cell, rotates, writes them back in cell order into the other buffer, and
// (when another step follows) streams and bins them for that step, so the
// particle data is read once and written once per step.
#pragma once

#include "mpcd_device.hpp"

namespace mpcd {

enum : uint32_t { ERR_STREAM_RANGE = 1u, ERR_FIXED_RANGE = 2u, ERR_GAMMA_CAP = 4u, ERR_LIST = 8u };

struct Box {
  int n[3];
  double L[3];
  double a, inv_a, dt;
  float a32, inv_a32, dt32;
  uint32_t ncells;
  double ca, sa, omc;  // cos(alpha), sin(alpha), 1 - cos(alpha)
  double kT, mass;
  uint32_t k0, k1;     // Philox key = user seed
  uint32_t n_solvent;
};

struct Particles {
  double* x[3];
  double* v[3];
  uint32_t* h;
  float* o[3];
  float* vf[3];
  uint32_t* tag;
};

// Blocks are handed to the 8 XCDs round-robin; remapping makes XCD k work on
// one contiguous range of cells so neighbouring cells share its L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u;
  const uint32_t x = b & 7u, i = b >> 3;
  return x < r ? x * (q + 1u) + i : r * (q + 1u) + (x - r) * q + i;
}

// ------------------------------------------------------------------ helpers
template <int FORM>
__device__ inline void load_vel(const Particles& P, uint32_t i, double v[3]) {
  if constexpr (FORM == 0) {
    v[0] = P.v[0][i];
    v[1] = P.v[1][i];
    v[2] = P.v[2][i];
  } else {
    v[0] = (double)P.vf[0][i];
    v[1] = (double)P.vf[1][i];
    v[2] = (double)P.vf[2][i];
  }
}

// Stream one particle (eq. 1) in place in registers.
// FP64: x <- wrap(x + v dt); FP32: offsets and home cells.
template <int FORM>
struct Pos;
template <>
struct Pos<0> {
  double x[3];
  __device__ void load(const Particles& P, uint32_t i) {
    x[0] = P.x[0][i];
    x[1] = P.x[1][i];
    x[2] = P.x[2][i];
  }
  __device__ void store(const Particles& P, uint32_t j) const {
    P.x[0][j] = x[0];
    P.x[1][j] = x[1];
    P.x[2][j] = x[2];
  }
  __device__ void stream(const Box& B, const double v[3], uint32_t& err) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double st = v[d] * B.dt;
      if (!(fabs(st) < B.L[d])) err |= ERR_STREAM_RANGE;
      x[d] = wrap_box(x[d] + st, B.L[d]);
    }
  }
  __device__ uint32_t cell(const Box& B, const double s[3], const float*) const {
    const int ix = bin_axis64(x[0], s[0], B.L[0], B.inv_a, B.n[0]);
    const int iy = bin_axis64(x[1], s[1], B.L[1], B.inv_a, B.n[1]);
    const int iz = bin_axis64(x[2], s[2], B.L[2], B.inv_a, B.n[2]);
    return (uint32_t)ix + (uint32_t)B.n[0] * ((uint32_t)iy + (uint32_t)B.n[1] * (uint32_t)iz);
  }
};
template <>
struct Pos<1> {
  int h[3];
  float o[3];
  __device__ void load(const Particles& P, uint32_t i) {
    unpack_home(P.h[i], h[0], h[1], h[2]);
    o[0] = P.o[0][i];
    o[1] = P.o[1][i];
    o[2] = P.o[2][i];
  }
  __device__ void store(const Particles& P, uint32_t j) const {
    P.h[j] = pack_home(h[0], h[1], h[2]);
    P.o[0][j] = o[0];
    P.o[1][j] = o[1];
    P.o[2][j] = o[2];
  }
  // v holds the velocity as stored (FP32 values)
  __device__ void stream(const Box& B, const double v[3], uint32_t&) {
#pragma unroll
    for (int d = 0; d < 3; ++d)
      stream_axis32(o[d], h[d], (float)v[d], B.dt32, B.a32, B.inv_a32, B.n[d]);
  }
  __device__ uint32_t cell(const Box& B, const double*, const float s32[3]) const {
    const int ix = bin_axis32(o[0], h[0], s32[0], B.inv_a32, B.n[0]);
    const int iy = bin_axis32(o[1], h[1], s32[1], B.inv_a32, B.n[1]);
    const int iz = bin_axis32(o[2], h[2], s32[2], B.inv_a32, B.n[2]);
    return (uint32_t)ix + (uint32_t)B.n[0] * ((uint32_t)iy + (uint32_t)B.n[1] * (uint32_t)iz);
  }
};

// ------------------------------------------------------- stream and bin
template <int FORM>
__global__ __launch_bounds__(256) void k_stream(Particles P, Box B, uint32_t N,
                                                uint32_t* err) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= N) return;
  double v[3];
  load_vel<FORM>(P, j, v);
  Pos<FORM> r;
  r.load(P, j);
  uint32_t e = 0;
  r.stream(B, v, e);
  r.store(P, j);
  if (e) atomicOr(err, e);
}

// Bin (optionally after streaming in place): collision cell on the shifted
// grid, and a rank inside the cell from one atomic per particle (count sort).
template <int FORM, bool STREAM>
__global__ __launch_bounds__(256) void k_bin(Particles P, Box B, uint32_t N,
                                             double s0, double s1, double s2,
                                             float t0, float t1, float t2,
                                             uint32_t* __restrict__ count,
                                             uint2* __restrict__ cr,
                                             uint32_t* err) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= N) return;
  Pos<FORM> r;
  r.load(P, j);
  if constexpr (STREAM) {
    double v[3];
    load_vel<FORM>(P, j, v);
    uint32_t e = 0;
    r.stream(B, v, e);
    r.store(P, j);
    if (e) atomicOr(err, e);
  }
  const double s[3] = {s0, s1, s2};
  const float s32[3] = {t0, t1, t2};
  const uint32_t c = r.cell(B, s, s32);
  const uint32_t rank = atomicAdd(&count[c], 1u);
  cr[j] = make_uint2(c, rank);
}

// ---------------------------------------------------------- count scan
constexpr int SCAN_T = 256;
constexpr int SCAN_PER = 16;
constexpr int SCAN_CHUNK = SCAN_T * SCAN_PER;

template <int NT>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t& total) {
  __shared__ uint32_t wsum[NT / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t wpre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint32_t s = wsum[w];
    wpre += (w < wid) ? s : 0u;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return wpre + incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_partial(const uint32_t* __restrict__ count,
                                                         uint32_t ncells,
                                                         uint32_t* __restrict__ partial) {
  const uint32_t base = blockIdx.x * (uint32_t)SCAN_CHUNK;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    const uint32_t c = base + (uint32_t)k * SCAN_T + threadIdx.x;
    if (c < ncells) s += count[c];
  }
  uint32_t tot;
  (void)block_exclusive_scan<SCAN_T>(s, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* partial, uint32_t nb) {
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nb; base += 1024u) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? partial[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024>(v, tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
}

// off[c] = exclusive prefix of count; count is cleared for the next binning.
__global__ __launch_bounds__(SCAN_T) void k_scan_final(uint32_t* __restrict__ count,
                                                       uint32_t ncells,
                                                       const uint32_t* __restrict__ partial,
                                                       uint32_t* __restrict__ off,
                                                       uint32_t N) {
  const uint32_t base = blockIdx.x * (uint32_t)SCAN_CHUNK + threadIdx.x * (uint32_t)SCAN_PER;
  uint32_t v[SCAN_PER];
  if (base + SCAN_PER <= ncells) {
    const uint4* p = reinterpret_cast<const uint4*>(count + base);
#pragma unroll
    for (int q = 0; q < SCAN_PER / 4; ++q) {
      const uint4 t = p[q];
      v[4 * q] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) v[k] = (base + k < ncells) ? count[base + k] : 0u;
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) s += v[k];
  uint32_t tot;
  uint32_t run = partial[blockIdx.x] + block_exclusive_scan<SCAN_T>(s, tot);
  if (base + SCAN_PER <= ncells) {
    uint4* o = reinterpret_cast<uint4*>(off + base);
    uint4* z = reinterpret_cast<uint4*>(count + base);
#pragma unroll
    for (int q = 0; q < SCAN_PER / 4; ++q) {
      uint4 t;
      t.x = run;
      run += v[4 * q];
      t.y = run;
      run += v[4 * q + 1];
      t.z = run;
      run += v[4 * q + 2];
      t.w = run;
      run += v[4 * q + 3];
      o[q] = t;
      z[q] = make_uint4(0u, 0u, 0u, 0u);
    }
  } else {
#pragma unroll
    for (int k = 0; k < SCAN_PER; ++k) {
      if (base + k < ncells) {
        off[base + k] = run;
        count[base + k] = 0u;
        run += v[k];
      }
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) off[ncells] = N;
}

// Cell-ordered particle list: perm[off[c] + rank] = current index.
__global__ __launch_bounds__(256) void k_perm(const uint2* __restrict__ cr,
                                              const uint32_t* __restrict__ off,
                                              uint32_t* __restrict__ perm, uint32_t N,
                                              uint32_t* err) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= N) return;
  const uint2 q = cr[i];
  const uint32_t j = off[q.x] + q.y;
  if (j < N) perm[j] = i;
  else atomicOr(err, ERR_LIST);
}

// ------------------------------------------------------------ per cell
// Cell sums (sec. 3.5, eq. 3): mass, momentum and, when asked, the kinetic
// energy relative to u, accumulated in exact fixed point. `get(k, v, m)`
// returns the velocity and mass of the cell's k-th particle.
struct CellSums {
  double M, u[3], ek;
};

template <bool EMB, bool EK, class Get>
__device__ inline CellSums cell_sums(uint32_t cnt, double solvent_mass, Get get,
                                     bool& bad) {
  CellSums r;
  Fx P[3] = {{0, 0}, {0, 0}, {0, 0}};
  Fx Mx = {0, 0};
  for (uint32_t k = 0; k < cnt; ++k) {
    double v[3], m;
    get(k, v, m);
    if constexpr (EMB) fx_add(Mx, m, bad);
    fx_add(P[0], m * v[0], bad);
    fx_add(P[1], m * v[1], bad);
    fx_add(P[2], m * v[2], bad);
  }
  r.M = EMB ? fx_value(Mx) : (double)cnt * solvent_mass;
  if (cnt > 0) {
    r.u[0] = fx_value(P[0]) / r.M;
    r.u[1] = fx_value(P[1]) / r.M;
    r.u[2] = fx_value(P[2]) / r.M;
  } else {
    r.u[0] = r.u[1] = r.u[2] = 0.0;
  }
  r.ek = 0.0;
  if constexpr (EK) {
    Fx E = {0, 0};
    for (uint32_t k = 0; k < cnt; ++k) {
      double v[3], m;
      get(k, v, m);
      const double dx = v[0] - r.u[0], dy = v[1] - r.u[1], dz = v[2] - r.u[2];
      fx_add(E, m * (dx * dx + dy * dy + dz * dz), bad);
    }
    r.ek = 0.5 * fx_value(E);
  }
  return r;
}

// --------------------------------------------------------------- collide
constexpr int COLLIDE_T = 256;
constexpr int PCAP = 1664;

struct CollideArgs {
  Particles cur, nxt;
  Box B;
  const uint32_t* off;
  const uint32_t* perm;
  const double* emb_mass;
  uint32_t step;      // counter of this collision
  uint32_t step_next; // counter of the following step (STREAM_NEXT)
  double sn[3];       // shift of the following step
  float sn32[3];
  uint32_t* count;    // occupancy of the following step (STREAM_NEXT)
  uint2* cr_next;
  uint32_t* err;
};

template <int FORM>
struct VelLds {
  using T = double;
};
template <>
struct VelLds<1> {
  using T = float;
};

template <int FORM, int CPB, bool STREAM_NEXT, bool THERMO, bool EMB>
__global__ __launch_bounds__(COLLIDE_T) void k_collide(CollideArgs A) {
  using VT = typename VelLds<FORM>::T;
  __shared__ VT s_v[3][PCAP];
  __shared__ uint32_t s_src[PCAP];
  __shared__ uint8_t s_lc[PCAP];
  __shared__ uint32_t s_tag[EMB ? PCAP : 1];
  __shared__ double s_u[3][CPB];
  __shared__ double s_R[9][CPB];
  __shared__ uint32_t s_off[CPB + 1];

  const Box& B = A.B;
  const uint32_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t c0 = blk * (uint32_t)CPB;
  const uint32_t nc = min((uint32_t)CPB, B.ncells - c0);
  const uint32_t tid = threadIdx.x;
  for (uint32_t t = tid; t <= nc; t += COLLIDE_T) s_off[t] = A.off[c0 + t];
  __syncthreads();
  const uint32_t s0 = s_off[0];
  const uint32_t np = s_off[nc] - s0;
  const uint32_t nlds = np < (uint32_t)PCAP ? np : (uint32_t)PCAP;

  // phase 1: stage the block's velocities (gathered through the list)
  for (uint32_t k = tid; k < nlds; k += COLLIDE_T) {
    const uint32_t i = A.perm[s0 + k];
    s_src[k] = i;
    if constexpr (FORM == 0) {
      s_v[0][k] = A.cur.v[0][i];
      s_v[1][k] = A.cur.v[1][i];
      s_v[2][k] = A.cur.v[2][i];
    } else {
      s_v[0][k] = A.cur.vf[0][i];
      s_v[1][k] = A.cur.vf[1][i];
      s_v[2][k] = A.cur.vf[2][i];
    }
    if constexpr (EMB) s_tag[k] = A.cur.tag[i];
  }
  __syncthreads();

  // phase 2: one thread per cell -> u, axis, xi, rotation matrix
  bool bad = false, cap = false;
  if (tid < nc) {
    const uint32_t b = s_off[tid] - s0, e = s_off[tid + 1] - s0;
    const uint32_t cnt = e - b;
    auto get = [&](uint32_t k, double v[3], double& m) {
      const uint32_t q = b + k;
      uint32_t tg;
      if (q < (uint32_t)PCAP) {
        v[0] = (double)s_v[0][q];
        v[1] = (double)s_v[1][q];
        v[2] = (double)s_v[2][q];
        if constexpr (EMB) tg = s_tag[q];
      } else {
        const uint32_t i = A.perm[s0 + q];
        load_vel<FORM>(A.cur, i, v);
        if constexpr (EMB) tg = A.cur.tag[i];
      }
      if constexpr (EMB)
        m = tg >= B.n_solvent ? A.emb_mass[tg - B.n_solvent] : B.mass;
      else
        m = B.mass;
    };
    const CellSums cs = cell_sums<EMB, THERMO>(cnt, B.mass, get, bad);
    for (uint32_t q = b; q < e && q < (uint32_t)PCAP; ++q) s_lc[q] = (uint8_t)tid;
    double n[3] = {0.0, 0.0, 0.0}, xi = 1.0;
    if (cnt > 0) {
      cell_axis(c0 + tid, A.step, B.k0, B.k1, n);
      if constexpr (THERMO) xi = thermo_xi(cnt, cs.ek, c0 + tid, A.step, B.k0, B.k1, B.kT, cap);
    }
    double R[9];
    rotation_matrix(n, B.ca, B.sa, B.omc, xi, R);
    s_u[0][tid] = cs.u[0];
    s_u[1][tid] = cs.u[1];
    s_u[2][tid] = cs.u[2];
#pragma unroll
    for (int q = 0; q < 9; ++q) s_R[q][tid] = R[q];
  }
  __syncthreads();

  // phase 3: rotate each particle (Alg. 1), write it in cell order; when a
  // step follows, stream it and count it into its next cell.
  uint32_t e = 0;
  for (uint32_t k = tid; k < np; k += COLLIDE_T) {
    uint32_t lc, i;
    double v[3];
    if (k < (uint32_t)PCAP) {
      lc = s_lc[k];
      i = s_src[k];
      v[0] = (double)s_v[0][k];
      v[1] = (double)s_v[1][k];
      v[2] = (double)s_v[2][k];
    } else {
      i = A.perm[s0 + k];
      load_vel<FORM>(A.cur, i, v);
      uint32_t lo = 0, hi = nc;  // last cell whose start <= s0 + k
      while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_off[mid] <= s0 + k) lo = mid; else hi = mid;
      }
      lc = lo;
    }
    const double ux = s_u[0][lc], uy = s_u[1][lc], uz = s_u[2][lc];
    const double dx = v[0] - ux, dy = v[1] - uy, dz = v[2] - uz;
    double w[3];
    w[0] = ux + (s_R[0][lc] * dx + s_R[1][lc] * dy + s_R[2][lc] * dz);
    w[1] = uy + (s_R[3][lc] * dx + s_R[4][lc] * dy + s_R[5][lc] * dz);
    w[2] = uz + (s_R[6][lc] * dx + s_R[7][lc] * dy + s_R[8][lc] * dz);
    const uint32_t j = s0 + k;
    if constexpr (FORM == 0) {
      A.nxt.v[0][j] = w[0];
      A.nxt.v[1][j] = w[1];
      A.nxt.v[2][j] = w[2];
    } else {
      const float f0 = (float)w[0], f1 = (float)w[1], f2 = (float)w[2];
      A.nxt.vf[0][j] = f0;
      A.nxt.vf[1][j] = f1;
      A.nxt.vf[2][j] = f2;
      w[0] = f0;
      w[1] = f1;
      w[2] = f2;
    }
    if constexpr (EMB)
      A.nxt.tag[j] = k < (uint32_t)PCAP ? s_tag[k] : A.cur.tag[i];
    else
      A.nxt.tag[j] = A.cur.tag[i];
    Pos<FORM> r;
    r.load(A.cur, i);
    if constexpr (STREAM_NEXT) {
      r.stream(B, w, e);
      const uint32_t c = r.cell(B, A.sn, A.sn32);
      const uint32_t rank = atomicAdd(&A.count[c], 1u);
      A.cr_next[j] = make_uint2(c, rank);
    }
    r.store(A.nxt, j);
  }
  if (bad) e |= ERR_FIXED_RANGE;
  if (cap) e |= ERR_GAMMA_CAP;
  if (e) atomicOr(A.err, e);
}

// ------------------------------------------------------- diagnostics
// Cell properties and draws of the binned state, one thread per cell,
// particles read through the cell-ordered list.
template <int FORM, bool THERMO, bool EMB>
__global__ __launch_bounds__(256) void k_cell_diag(Particles P, Box B,
                                                   const uint32_t* __restrict__ off,
                                                   const uint32_t* __restrict__ perm,
                                                   const double* __restrict__ emb_mass,
                                                   uint32_t step, double* mass,
                                                   double* ek,
                                                   double* axis, double* xi_out,
                                                   uint32_t* err) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= B.ncells) return;
  const uint32_t b = off[c], cnt = off[c + 1] - b;
  auto get = [&](uint32_t k, double v[3], double& m) {
    const uint32_t i = perm[b + k];
    load_vel<FORM>(P, i, v);
    if constexpr (EMB) {
      const uint32_t tg = P.tag[i];
      m = tg >= B.n_solvent ? emb_mass[tg - B.n_solvent] : B.mass;
    } else {
      m = B.mass;
    }
  };
  bool bad = false, cap = false;
  const CellSums cs = cell_sums<EMB, true>(cnt, B.mass, get, bad);
  mass[c] = cs.M;
  ek[c] = cs.ek;
  double n[3] = {0.0, 0.0, 0.0}, xi = 1.0;
  if (cnt > 0) {
    cell_axis(c, step, B.k0, B.k1, n);
    if constexpr (THERMO) xi = thermo_xi(cnt, cs.ek, c, step, B.k0, B.k1, B.kT, cap);
  }
  axis[3 * c] = n[0];
  axis[3 * c + 1] = n[1];
  axis[3 * c + 2] = n[2];
  xi_out[c] = xi;
  uint32_t e = (bad ? ERR_FIXED_RANGE : 0u) | (cap ? ERR_GAMMA_CAP : 0u);
  if (e) atomicOr(err, e);
}

// Cell momentum for the diagnostics: the fixed-point sum itself.
template <int FORM, bool EMB>
__global__ __launch_bounds__(256) void k_cell_momentum(Particles P, Box B,
                                                       const uint32_t* __restrict__ off,
                                                       const uint32_t* __restrict__ perm,
                                                       const double* __restrict__ emb_mass,
                                                       double* mom, uint32_t* err) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= B.ncells) return;
  const uint32_t b = off[c], cnt = off[c + 1] - b;
  Fx S[3] = {{0, 0}, {0, 0}, {0, 0}};
  bool bad = false;
  for (uint32_t k = 0; k < cnt; ++k) {
    const uint32_t i = perm[b + k];
    double v[3];
    load_vel<FORM>(P, i, v);
    double m = B.mass;
    if constexpr (EMB) {
      const uint32_t tg = P.tag[i];
      if (tg >= B.n_solvent) m = emb_mass[tg - B.n_solvent];
    }
    fx_add(S[0], m * v[0], bad);
    fx_add(S[1], m * v[1], bad);
    fx_add(S[2], m * v[2], bad);
  }
  mom[3 * c] = fx_value(S[0]);
  mom[3 * c + 1] = fx_value(S[1]);
  mom[3 * c + 2] = fx_value(S[2]);
  if (bad) atomicOr(err, ERR_FIXED_RANGE);
}

// Net momentum, kinetic energy and mass in fixed point: block sums in LDS
// (integer, so exact), then 64-bit atomics, which commute.
template <int FORM, bool EMB>
__global__ __launch_bounds__(256) void k_totals(Particles P, Box B, uint32_t N,
                                                const double* __restrict__ emb_mass,
                                                long long* tot, uint32_t* err) {
  __shared__ long long red[10][256];
  Fx acc[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  bool bad = false;
  for (uint32_t j = blockIdx.x * 256u + threadIdx.x; j < N; j += gridDim.x * 256u) {
    double v[3];
    load_vel<FORM>(P, j, v);
    double m = B.mass;
    if constexpr (EMB) {
      const uint32_t tg = P.tag[j];
      if (tg >= B.n_solvent) m = emb_mass[tg - B.n_solvent];
    }
    fx_add(acc[0], m * v[0], bad);
    fx_add(acc[1], m * v[1], bad);
    fx_add(acc[2], m * v[2], bad);
    fx_add(acc[3], m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]), bad);
    fx_add(acc[4], m, bad);
  }
  for (int q = 0; q < 5; ++q) {
    red[2 * q][threadIdx.x] = acc[q].hi;
    red[2 * q + 1][threadIdx.x] = acc[q].lo;
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 10; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 10)
    atomicAdd(reinterpret_cast<unsigned long long*>(&tot[threadIdx.x]),
              (unsigned long long)red[threadIdx.x][0]);
  if (bad) atomicOr(err, ERR_FIXED_RANGE);
}

// ------------------------------------------------------------ state I/O
// Row-major N x 3 doubles (tag order) -> internal layout; checks the box.
template <int FORM>
__global__ __launch_bounds__(256) void k_import(Particles P, Box B,
                                                const double* __restrict__ pos,
                                                const double* __restrict__ vel,
                                                uint32_t n, uint32_t tag0,
                                                uint32_t* bad_pos) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= n) return;
  const uint32_t j = tag0 + t;
  double x[3], v[3];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d] = pos[3ull * t + d];
    v[d] = vel[3ull * t + d];
    bad |= !(x[d] >= 0.0 && x[d] < B.L[d]);
  }
  if (bad) atomicOr(bad_pos, 1u);
  if constexpr (FORM == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      P.x[d][j] = x[d];
      P.v[d][j] = v[d];
    }
  } else {
    int h[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int hd = (int)floor(x[d] * B.inv_a);
      hd = hd < 0 ? 0 : (hd > B.n[d] - 1 ? B.n[d] - 1 : hd);
      float o = (float)(x[d] - (double)hd * B.a);
      if (o >= B.a32) {
        o = 0.0f;
        hd = hd + 1 == B.n[d] ? 0 : hd + 1;
      }
      if (o < 0.0f) o = 0.0f;
      h[d] = hd;
      P.o[d][j] = o;
      P.vf[d][j] = (float)v[d];
    }
    P.h[j] = pack_home(h[0], h[1], h[2]);
  }
  P.tag[j] = j;
}

// Internal layout -> row-major N x 3 doubles in tag order.
template <int FORM>
__global__ __launch_bounds__(256) void k_export(Particles P, Box B, uint32_t N,
                                                double* __restrict__ pos,
                                                double* __restrict__ vel) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= N) return;
  const uint32_t t = P.tag[j];
  if constexpr (FORM == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pos[3ull * t + d] = P.x[d][j];
      vel[3ull * t + d] = P.v[d][j];
    }
  } else {
    int h[3];
    unpack_home(P.h[j], h[0], h[1], h[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pos[3ull * t + d] = (double)h[d] * B.a + (double)P.o[d][j];
      vel[3ull * t + d] = (double)P.vf[d][j];
    }
  }
}

// Cells of the last binning in tag order: from (cell, rank) of the current
// order, or, after a collide, from the cell-ordered layout itself.
__global__ __launch_bounds__(256) void k_cells_from_cr(const uint32_t* __restrict__ tag,
                                                       const uint2* __restrict__ cr,
                                                       uint32_t N, int32_t* out) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= N) return;
  out[tag[j]] = (int32_t)cr[j].x;
}

__global__ __launch_bounds__(256) void k_cells_from_order(const uint32_t* __restrict__ tag,
                                                          const uint32_t* __restrict__ off,
                                                          uint32_t ncells, int32_t* out,
                                                          int32_t* counts) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= ncells) return;
  const uint32_t b = off[c], e = off[c + 1];
  if (counts) counts[c] = (int32_t)(e - b);
  if (out)
    for (uint32_t j = b; j < e; ++j) out[tag[j]] = (int32_t)c;
}

// --------------------------------------------------------- test kernels
__global__ void k_philox(const U4* __restrict__ ctr, uint32_t n, uint32_t k0,
                         uint32_t k1, U4* __restrict__ out) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

// Streaming copy, 16-byte vectors, grid-stride.
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * 256u + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * 256u)
    dst[i] = src[i];
}

__global__ void k_copy1(const unsigned char* __restrict__ src,
                        unsigned char* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace mpcd
