// Kernels of the SRD step on gfx950 (wave64, 160 KB LDS per CU, 8 XCDs).
//
// Data layout in HBM. The box is cut into tiles of td[0] x td[1] x td[2]
// cells (4x4x4 or 4x4x8). Every tile owns a slab of `cap` particle slots in
// each of two buffers; the first cnt[T] slots of tile T hold its particles in
// no particular order. Within a slab the data is structure of arrays, one
// array per component, so a block reads and writes its tile as unit-stride
// streams:
//   FP64 form: x[3][S], v[3][S] double;
//   FP32 form: h[S] home cell packed 10:10:10, o[3][S] float offset inside the
//              home cell, v[3][S] float;
//   tag[S] uint32 particle identity;            S = ntiles * cap.
//
// One step is one launch of k_tile: block T gathers its tile (binned for this
// step: every particle's collision cell lies in T), sums each cell exactly in
// LDS, draws the cell's axis and thermostat factor, rotates, then streams the
// particles, bins them for the next step's shift and scatters them to the
// next tile's slab in the other buffer. Destination slots are reserved with
// one global atomic per (block, destination tile) pair -- at most 27 per
// block -- so the particle data is read once and written once per step and
// no per-particle global atomics are needed.
#pragma once

#include "mpcd_device.hpp"

namespace mpcd {

enum : uint32_t {
  ERR_STREAM_RANGE = 1u,  // |v dt| >= L in the FP64 form
  ERR_FIXED_RANGE = 2u,   // a term outside the fixed-point range
  ERR_GAMMA_CAP = 4u,     // Gamma sampler reached its attempt cap
  ERR_TILE = 8u,          // a particle was found outside its tile (a bug)
};

// status[0]: error flags above; status[1]: nonzero once a slab overflowed;
// status[2]: smallest launch sequence number that overflowed (tile kernels
// with a larger sequence number return at once).
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
  int td[3];           // tile size in cells
  int tsh[3];          // log2(td) (td is a power of two whenever nt > 1)
  int nt[3];           // tiles per axis
  uint32_t ntiles;
  uint32_t cap;        // slots per tile
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
// one contiguous range of tiles, so neighbouring tiles share its L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u;
  const uint32_t x = b & 7u, i = b >> 3;
  return x < r ? x * (q + 1u) + i : r * (q + 1u) + (x - r) * q + i;
}

__device__ inline int tile_coord(int c, const Box& B, int d) {
  return B.nt[d] == 1 ? 0 : (c >> B.tsh[d]);
}

template <int FORM>
struct VelT {
  using T = double;
};
template <>
struct VelT<1> {
  using T = float;
};

template <int FORM>
__device__ inline void load_vel(const Particles& P, size_t i, double v[3]) {
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

template <int FORM>
__device__ inline void store_vel(const Particles& P, size_t j, const double w[3]) {
  if constexpr (FORM == 0) {
    P.v[0][j] = w[0];
    P.v[1][j] = w[1];
    P.v[2][j] = w[2];
  } else {
    P.vf[0][j] = (float)w[0];
    P.vf[1][j] = (float)w[1];
    P.vf[2][j] = (float)w[2];
  }
}

// Position of one particle in registers: stream (eq. 1) and bin (sec. 3.4).
template <int FORM>
struct Pos;
template <>
struct Pos<0> {
  double x[3];
  __device__ void load(const Particles& P, size_t i) {
    x[0] = P.x[0][i];
    x[1] = P.x[1][i];
    x[2] = P.x[2][i];
  }
  __device__ void store(const Particles& P, size_t j) const {
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
  __device__ void cell3(const Box& B, const double s[3], const float*, int c[3]) const {
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = bin_axis64(x[d], s[d], B.L[d], B.inv_a, B.n[d]);
  }
  __device__ void home3(const Box& B, int c[3]) const {
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = bin_axis64(x[d], 0.0, B.L[d], B.inv_a, B.n[d]);
  }
};
template <>
struct Pos<1> {
  int h[3];
  float o[3];
  __device__ void load(const Particles& P, size_t i) {
    unpack_home(P.h[i], h[0], h[1], h[2]);
    o[0] = P.o[0][i];
    o[1] = P.o[1][i];
    o[2] = P.o[2][i];
  }
  __device__ void store(const Particles& P, size_t j) const {
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
  __device__ void cell3(const Box& B, const double*, const float s32[3], int c[3]) const {
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = bin_axis32(o[d], h[d], s32[d], B.inv_a32, B.n[d]);
  }
  __device__ void home3(const Box&, int c[3]) const {
    c[0] = h[0];
    c[1] = h[1];
    c[2] = h[2];
  }
};

__device__ inline uint32_t cell_index(const Box& B, const int c[3]) {
  return (uint32_t)c[0] + (uint32_t)B.n[0] * ((uint32_t)c[1] + (uint32_t)B.n[1] * (uint32_t)c[2]);
}

__device__ inline uint32_t tile_index(const Box& B, const int c[3]) {
  const int tx = tile_coord(c[0], B, 0), ty = tile_coord(c[1], B, 1), tz = tile_coord(c[2], B, 2);
  return (uint32_t)tx + (uint32_t)B.nt[0] * ((uint32_t)ty + (uint32_t)B.nt[1] * (uint32_t)tz);
}

// ------------------------------------------------------- scatter helpers
// Destination bin of a particle leaving tile t for the tile of cell c:
// 0..26 for the 27 neighbours (periodic wrap), 27 for any other tile.
__device__ inline uint32_t dest_bin(const Box& B, const int t[3], const int c[3]) {
  uint32_t bin = 0, mul = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int nt = B.nt[d];
    const int ct = tile_coord(c[d], B, d);
    int o;
    if (ct == t[d]) o = 1;
    else if (ct == (t[d] + 1 == nt ? 0 : t[d] + 1)) o = 2;
    else if (ct == (t[d] == 0 ? nt - 1 : t[d] - 1)) o = 0;
    else return 27u;
    bin += (uint32_t)o * mul;
    mul *= 3u;
  }
  return bin;
}

__device__ inline uint32_t bin_tile(const Box& B, const int t[3], uint32_t bin) {
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int o = (int)(bin % 3u) - 1;
    bin /= 3u;
    int x = t[d] + o;
    if (x < 0) x += B.nt[d];
    if (x >= B.nt[d]) x -= B.nt[d];
    c[d] = x;
  }
  return (uint32_t)c[0] + (uint32_t)B.nt[0] * ((uint32_t)c[1] + (uint32_t)B.nt[1] * (uint32_t)c[2]);
}

// Rank of each active lane among the block's particles with the same bin:
// lanes of one wave are ranked in lane order (ballot), waves take
// consecutive ranges through one LDS atomic per (wave, bin).
__device__ inline uint32_t wave_rank(uint32_t bin, bool active, uint32_t* s_bincnt) {
  const uint32_t lane = threadIdx.x & 63u;
  unsigned long long pending = __ballot(active);
  uint32_t myrank = 0;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const uint32_t b = __shfl(bin, leader);
    const unsigned long long m = __ballot(active && bin == b);
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(&s_bincnt[b], (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (active && bin == b) myrank = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    pending &= ~m;
  }
  return myrank;
}

// ------------------------------------------------------------ tile kernel
enum { MODE_BIN = 0, MODE_COLLIDE = 1, MODE_COLLIDE_SCATTER = 2, MODE_DIAG = 3 };

constexpr int TT = 256;         // threads per tile block
constexpr int TQ = 4;           // particles per thread held in registers
constexpr int TREG = TT * TQ;   // beyond this a tile's particles are re-read

struct TileArgs {
  Particles in, out;
  Box B;
  const uint32_t* cnt_in;   // occupancy of the input slabs
  uint32_t* cnt_out;        // occupancy of the output slabs (scatter modes)
  uint32_t* cnt_clear;      // cleared for this tile (scatter modes)
  const double* emb_mass;
  uint32_t step;            // counter of the collision
  double s[3];              // shift binning the input (collide) or output (bin)
  float s32[3];
  double sn[3];             // shift of the next step (collide + scatter)
  float sn32[3];
  uint32_t* status;
  uint32_t seq;             // launch sequence number within one API call
  double* d_mass;           // per-cell outputs of MODE_DIAG (global cell index)
  double* d_mom;
  double* d_ek;
  double* d_axis;
  double* d_xi;
};

template <int FORM, int CPT, int MODE, bool STREAM_IN, bool THERMO, bool EMB>
__global__ __launch_bounds__(TT) void k_tile(TileArgs A) {
  using VT = typename VelT<FORM>::T;
  constexpr bool COLL = MODE != MODE_BIN;
  constexpr bool SCAT = MODE == MODE_BIN || MODE == MODE_COLLIDE_SCATTER;
  constexpr bool EK = THERMO || MODE == MODE_DIAG;
  constexpr int TPC = TT / CPT;  // threads per cell in the per-cell phase
  // accumulator rows: 0 count, 1..6 momentum limbs, then energy, then mass
  constexpr int IE = 7;
  constexpr int IM = EK ? 9 : 7;
  constexpr int NACC = COLL ? (IM + (EMB ? 2 : 0)) : 1;
  constexpr int CC = COLL ? CPT : 1;
  __shared__ unsigned long long s_acc[NACC][CC];
  __shared__ double s_u[3][CC];
  __shared__ double s_R[9][CC];
  __shared__ double s_g[THERMO ? TPC : 1][THERMO ? CPT : 1];
  __shared__ uint32_t s_bincnt[28];
  __shared__ uint32_t s_base[28];
  __shared__ uint32_t s_quit;

  const Box& B = A.B;
  const uint32_t tid = threadIdx.x;
  // quit if an earlier launch of this call overflowed a slab (launches of
  // the failing one itself run to the end, so its counts are complete)
  if (tid == 0) s_quit = (A.status[1] != 0u && A.status[2] < A.seq) ? 1u : 0u;
  if (tid < 28u) s_bincnt[tid] = 0u;
  if constexpr (COLL)
    for (uint32_t t = tid; t < (uint32_t)(NACC * CC); t += TT) (&s_acc[0][0])[t] = 0ull;
  __syncthreads();
  if (s_quit) return;

  const uint32_t T = xcd_remap(blockIdx.x, gridDim.x);
  int t3[3];
  t3[0] = (int)(T % (uint32_t)B.nt[0]);
  t3[1] = (int)((T / (uint32_t)B.nt[0]) % (uint32_t)B.nt[1]);
  t3[2] = (int)(T / ((uint32_t)B.nt[0] * (uint32_t)B.nt[1]));
  int org[3], ext[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    org[d] = t3[d] * B.td[d];
    ext[d] = min(B.td[d], B.n[d] - org[d]);
  }
  const uint32_t cnt = min(A.cnt_in[T], B.cap);
  const uint32_t nreg = min(cnt, (uint32_t)TREG);
  const size_t base_in = (size_t)T * B.cap;
  if (SCAT && tid == 0 && A.cnt_clear) A.cnt_clear[T] = 0u;

  uint32_t err = 0;
  bool bad = false, cap = false;

  auto mass_of = [&](uint32_t tag) -> double {
    if constexpr (EMB) return tag >= B.n_solvent ? A.emb_mass[tag - B.n_solvent] : B.mass;
    else return B.mass;
  };
  // local cell (inside this tile) of a particle binned with the input shift
  auto local_cell = [&](const Pos<FORM>& r) -> uint32_t {
    int c[3];
    r.cell3(B, A.s, A.s32, c);
    int l[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      l[d] = c[d] - org[d];
      if (l[d] < 0 || l[d] >= ext[d]) {
        err |= ERR_TILE;
        l[d] = l[d] < 0 ? 0 : ext[d] - 1;
      }
    }
    return (uint32_t)l[0] + (uint32_t)B.td[0] * ((uint32_t)l[1] + (uint32_t)B.td[1] * (uint32_t)l[2]);
  };
  auto add2 = [&](int j, uint32_t lc, double x) {
    long long hi, lo;
    fx_split(x, hi, lo, bad);
    atomicAdd(&s_acc[j][lc], (unsigned long long)hi);
    atomicAdd(&s_acc[j + 1][lc], (unsigned long long)lo);
  };
  auto acc_val = [&](int j, uint32_t lc) {
    Fx f;
    f.hi = (long long)s_acc[j][lc];
    f.lo = (long long)s_acc[j + 1][lc];
    return fx_value(f);
  };

  // per-cell work is done by TPC threads per cell: cell l, sub-thread sub
  const uint32_t l = tid / (uint32_t)TPC, sub = tid % (uint32_t)TPC;
  int lc3[3];
  lc3[0] = (int)(l % (uint32_t)B.td[0]);
  lc3[1] = (int)((l / (uint32_t)B.td[0]) % (uint32_t)B.td[1]);
  lc3[2] = (int)(l / ((uint32_t)B.td[0] * (uint32_t)B.td[1]));
  const bool cell_ok = l < (uint32_t)CPT && lc3[0] < ext[0] && lc3[1] < ext[1] && lc3[2] < ext[2];
  const int gc3[3] = {org[0] + lc3[0], org[1] + lc3[1], org[2] + lc3[2]};
  const uint32_t gcell = cell_ok ? cell_index(B, gc3) : 0u;

  // ---- gather this tile's particles (register-resident part)
  VT v[TQ][3];
  uint32_t tg[TQ];
  uint32_t lcs[TQ];
  Pos<FORM> r[TQ];
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const uint32_t k = tid + (uint32_t)(q * TT);
    lcs[q] = 0u;
    tg[q] = 0u;
    if (k < nreg) {
      const size_t i = base_in + k;
      if constexpr (FORM == 0) {
        v[q][0] = A.in.v[0][i];
        v[q][1] = A.in.v[1][i];
        v[q][2] = A.in.v[2][i];
      } else {
        v[q][0] = A.in.vf[0][i];
        v[q][1] = A.in.vf[1][i];
        v[q][2] = A.in.vf[2][i];
      }
      tg[q] = A.in.tag[i];
      r[q].load(A.in, i);
    }
  }

  // the cell's rotation axis needs only (cell, step): draw it while the
  // gathers are in flight
  double n[3] = {0.0, 0.0, 0.0};
  if constexpr (COLL)
    if (sub == 0u && cell_ok) cell_axis(gcell, A.step, B.k0, B.k1, n);

  // ---- scatter: bin for the destination shift, reserve slots, write
  auto scatter = [&](const double* sd, const float* sd32, const double (*w)[3]) {
    // w[q]: velocity to store (already rounded to the storage precision)
    uint32_t bins[TQ], ranks[TQ], dest[TQ];
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const uint32_t k = tid + (uint32_t)(q * TT);
      const bool act = k < nreg;
      uint32_t b = 0;
      dest[q] = 0u;
      if (act) {
        int c[3];
        r[q].cell3(B, sd, sd32, c);
        b = dest_bin(B, t3, c);
        dest[q] = b < 27u ? bin_tile(B, t3, b) : tile_index(B, c);
      }
      bins[q] = b;
      ranks[q] = (act && b < 27u) ? atomicAdd(&s_bincnt[b], 1u) : 0u;
    }
    __syncthreads();
    if (tid < 27u && s_bincnt[tid] > 0u)
      s_base[tid] = atomicAdd(&A.cnt_out[bin_tile(B, t3, tid)], s_bincnt[tid]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const uint32_t k = tid + (uint32_t)(q * TT);
      if (k < nreg) {
        const uint32_t slot = bins[q] < 27u ? s_base[bins[q]] + ranks[q]
                                            : atomicAdd(&A.cnt_out[dest[q]], 1u);
        if (slot < B.cap) {
          const size_t j = (size_t)dest[q] * B.cap + slot;
          store_vel<FORM>(A.out, j, w[q]);
          A.out.tag[j] = tg[q];
          r[q].store(A.out, j);
        } else {
          atomicMax(&A.status[1], 1u);
          atomicMin(&A.status[2], A.seq);
        }
      }
    }
  };
  // particles beyond the register-resident part: one global atomic each
  auto scatter_one = [&](Pos<FORM>& rr, const double* sd, const float* sd32, const double w[3],
                         uint32_t tag) {
    int c[3];
    rr.cell3(B, sd, sd32, c);
    const uint32_t dt = tile_index(B, c);
    const uint32_t slot = atomicAdd(&A.cnt_out[dt], 1u);
    if (slot < B.cap) {
      const size_t j = (size_t)dt * B.cap + slot;
      store_vel<FORM>(A.out, j, w);
      A.out.tag[j] = tag;
      rr.store(A.out, j);
    } else {
      atomicMax(&A.status[1], 1u);
      atomicMin(&A.status[2], A.seq);
    }
  };

  if constexpr (MODE == MODE_BIN) {
    double w[TQ][3];
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      w[q][0] = (double)v[q][0];
      w[q][1] = (double)v[q][1];
      w[q][2] = (double)v[q][2];
      if (STREAM_IN && tid + (uint32_t)(q * TT) < nreg) r[q].stream(B, w[q], err);
    }
    scatter(A.s, A.s32, w);
    for (uint32_t k = TREG + tid; k < cnt; k += TT) {
      const size_t i = base_in + k;
      double vv[3];
      load_vel<FORM>(A.in, i, vv);
      Pos<FORM> rr;
      rr.load(A.in, i);
      if (STREAM_IN) rr.stream(B, vv, err);
      scatter_one(rr, A.s, A.s32, vv, A.in.tag[i]);
    }
  } else {
    // ---- cell sums: count, momentum (and mass) in exact fixed point
    auto sum_mom = [&](uint32_t lc, const double vv[3], double m) {
      atomicAdd(&s_acc[0][lc], 1ull);
      add2(1, lc, m * vv[0]);
      add2(3, lc, m * vv[1]);
      add2(5, lc, m * vv[2]);
      if constexpr (EMB) add2(IM, lc, m);
    };
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const uint32_t k = tid + (uint32_t)(q * TT);
      if (k < nreg) {
        lcs[q] = local_cell(r[q]);
        const double vv[3] = {(double)v[q][0], (double)v[q][1], (double)v[q][2]};
        sum_mom(lcs[q], vv, mass_of(tg[q]));
      }
    }
    for (uint32_t k = TREG + tid; k < cnt; k += TT) {
      const size_t i = base_in + k;
      double vv[3];
      load_vel<FORM>(A.in, i, vv);
      Pos<FORM> rr;
      rr.load(A.in, i);
      sum_mom(local_cell(rr), vv, mass_of(A.in.tag[i]));
    }
    __syncthreads();

    // ---- per cell: u on sub-thread 0; Gamma attempts in parallel
    // (attempt j on sub-thread j; the first accepted one in attempt order is
    // the draw, exactly as when the attempts are made one after another)
    const uint32_t nc = cell_ok ? (uint32_t)s_acc[0][l] : 0u;
    if (nc == 0u) n[0] = n[1] = n[2] = 0.0;
    if (sub == 0u) {
      double u[3] = {0.0, 0.0, 0.0};
      if (nc > 0u) {
        const double M = EMB ? acc_val(IM, l) : (double)nc * B.mass;
        u[0] = acc_val(1, l) / M;
        u[1] = acc_val(3, l) / M;
        u[2] = acc_val(5, l) / M;
      }
      if (l < (uint32_t)CPT) {
        s_u[0][l] = u[0];
        s_u[1][l] = u[1];
        s_u[2][l] = u[2];
      }
    }
    if constexpr (THERMO) {
      if (l < (uint32_t)CPT) {
        double g = -1.0;  // -1: rejected or not drawn
        if (nc >= 2u) {
          const double k = 1.5 * (double)(nc - 1u);
          const double d = k - 1.0 / 3.0;
          g = gamma_attempt(gcell, A.step, sub, d, 1.0 / sqrt(9.0 * d), B.kT, B.k0, B.k1);
        }
        s_g[sub][l] = g;
      }
    }
    __syncthreads();

    if constexpr (EK) {
      auto sum_energy = [&](uint32_t lc, const double vv[3], double m) {
        const double dx = vv[0] - s_u[0][lc], dy = vv[1] - s_u[1][lc], dz = vv[2] - s_u[2][lc];
        add2(IE, lc, m * (dx * dx + dy * dy + dz * dz));
      };
#pragma unroll
      for (int q = 0; q < TQ; ++q) {
        const uint32_t k = tid + (uint32_t)(q * TT);
        if (k < nreg) {
          const double vv[3] = {(double)v[q][0], (double)v[q][1], (double)v[q][2]};
          sum_energy(lcs[q], vv, mass_of(tg[q]));
        }
      }
      for (uint32_t k = TREG + tid; k < cnt; k += TT) {
        const size_t i = base_in + k;
        double vv[3];
        load_vel<FORM>(A.in, i, vv);
        Pos<FORM> rr;
        rr.load(A.in, i);
        sum_energy(local_cell(rr), vv, mass_of(A.in.tag[i]));
      }
      __syncthreads();
    }

    // ---- per cell: xi and the scaled rotation matrix (sub-thread 0)
    if (sub == 0u && l < (uint32_t)CPT) {
      double xi = 1.0;
      double ek = 0.0;
      if constexpr (EK) ek = 0.5 * acc_val(IE, l);
      if constexpr (THERMO) {
        if (nc >= 2u && ek > 0.0) {
          double ehat = -1.0;
          for (uint32_t j = 0; j < (uint32_t)TPC && ehat < 0.0; ++j) ehat = s_g[j][l];
          if (ehat < 0.0)  // every speculative attempt was rejected
            ehat = gamma_mt(1.5 * (double)(nc - 1u), gcell, A.step, B.k0, B.k1, B.kT, cap, TPC);
          xi = sqrt(ehat / ek);
        }
      }
      if constexpr (MODE == MODE_DIAG) {
        if (cell_ok) {
          A.d_mass[gcell] = nc > 0u ? (EMB ? acc_val(IM, l) : (double)nc * B.mass) : 0.0;
          A.d_mom[3u * gcell] = acc_val(1, l);
          A.d_mom[3u * gcell + 1u] = acc_val(3, l);
          A.d_mom[3u * gcell + 2u] = acc_val(5, l);
          A.d_ek[gcell] = ek;
          A.d_axis[3u * gcell] = n[0];
          A.d_axis[3u * gcell + 1u] = n[1];
          A.d_axis[3u * gcell + 2u] = n[2];
          A.d_xi[gcell] = xi;
        }
      } else {
        double R[9];
        rotation_matrix(n, B.ca, B.sa, B.omc, xi, R);
#pragma unroll
        for (int q = 0; q < 9; ++q) s_R[q][l] = R[q];
      }
    }

    if constexpr (MODE != MODE_DIAG) {
      __syncthreads();
      // ---- rotate (Alg. 1): v <- u + xi R (v - u), FP64 registers
      auto rotate = [&](uint32_t lc, const double vv[3], double w[3]) {
        const double ux = s_u[0][lc], uy = s_u[1][lc], uz = s_u[2][lc];
        const double dx = vv[0] - ux, dy = vv[1] - uy, dz = vv[2] - uz;
        w[0] = ux + (s_R[0][lc] * dx + s_R[1][lc] * dy + s_R[2][lc] * dz);
        w[1] = uy + (s_R[3][lc] * dx + s_R[4][lc] * dy + s_R[5][lc] * dz);
        w[2] = uz + (s_R[6][lc] * dx + s_R[7][lc] * dy + s_R[8][lc] * dz);
        if constexpr (FORM == 1) {
          w[0] = (double)(float)w[0];
          w[1] = (double)(float)w[1];
          w[2] = (double)(float)w[2];
        }
      };
      double w[TQ][3];
#pragma unroll
      for (int q = 0; q < TQ; ++q) {
        const uint32_t k = tid + (uint32_t)(q * TT);
        if (k < nreg) {
          const double vv[3] = {(double)v[q][0], (double)v[q][1], (double)v[q][2]};
          rotate(lcs[q], vv, w[q]);
          if constexpr (MODE == MODE_COLLIDE) {
            const size_t j = base_in + k;
            store_vel<FORM>(A.out, j, w[q]);
            A.out.tag[j] = tg[q];
            r[q].store(A.out, j);
          } else {
            r[q].stream(B, w[q], err);
          }
        }
      }
      if constexpr (MODE == MODE_COLLIDE_SCATTER) scatter(A.sn, A.sn32, w);
      for (uint32_t k = TREG + tid; k < cnt; k += TT) {
        const size_t i = base_in + k;
        double vv[3], ww[3];
        load_vel<FORM>(A.in, i, vv);
        Pos<FORM> rr;
        rr.load(A.in, i);
        rotate(local_cell(rr), vv, ww);
        if constexpr (MODE == MODE_COLLIDE) {
          store_vel<FORM>(A.out, i, ww);
          A.out.tag[i] = A.in.tag[i];
          rr.store(A.out, i);
        } else {
          rr.stream(B, ww, err);
          scatter_one(rr, A.sn, A.sn32, ww, A.in.tag[i]);
        }
      }
    }
  }
  if (bad) err |= ERR_FIXED_RANGE;
  if (cap) err |= ERR_GAMMA_CAP;
  if (err) atomicOr(&A.status[0], err);
}

// ------------------------------------------------- elementwise over slabs
// Valid slot k of tile T: k < cnt[T]. Grid: ntiles * ceil(cap / 256) blocks.
struct SlabIter {
  uint32_t T, k;
  size_t i;
  bool valid;
};
__device__ inline SlabIter slab_slot(const Box& B, const uint32_t* cnt) {
  const uint32_t per = (B.cap + 255u) / 256u;
  SlabIter s;
  s.T = blockIdx.x / per;
  s.k = (blockIdx.x % per) * 256u + threadIdx.x;
  s.i = (size_t)s.T * B.cap + s.k;
  s.valid = s.T < B.ntiles && s.k < min(cnt[s.T], B.cap);
  return s;
}

template <int FORM>
__global__ __launch_bounds__(256) void k_stream(Particles P, Box B, const uint32_t* cnt,
                                                uint32_t* status) {
  const SlabIter s = slab_slot(B, cnt);
  if (!s.valid) return;
  double v[3];
  load_vel<FORM>(P, s.i, v);
  Pos<FORM> r;
  r.load(P, s.i);
  uint32_t e = 0;
  r.stream(B, v, e);
  r.store(P, s.i);
  if (e) atomicOr(&status[0], e);
}

// Cell of every particle for shift s, in tag order, and the occupancy.
template <int FORM>
__global__ __launch_bounds__(256) void k_cells(Particles P, Box B, const uint32_t* cnt,
                                               double s0, double s1, double s2, float t0,
                                               float t1, float t2, int32_t* cell_of_tag,
                                               uint32_t* counts) {
  const SlabIter s = slab_slot(B, cnt);
  if (!s.valid) return;
  Pos<FORM> r;
  r.load(P, s.i);
  const double sd[3] = {s0, s1, s2};
  const float s32[3] = {t0, t1, t2};
  int c[3];
  r.cell3(B, sd, s32, c);
  const uint32_t cell = cell_index(B, c);
  if (cell_of_tag) cell_of_tag[P.tag[s.i]] = (int32_t)cell;
  if (counts) atomicAdd(&counts[cell], 1u);
}

// Net momentum, kinetic energy and mass in fixed point: block sums in LDS
// (integer, so exact), then 64-bit atomics, which commute.
template <int FORM, bool EMB>
__global__ __launch_bounds__(256) void k_totals(Particles P, Box B, const uint32_t* cnt,
                                                const double* __restrict__ emb_mass,
                                                long long* tot, uint32_t* status) {
  __shared__ long long red[10][256];
  Fx acc[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  bool bad = false;
  const SlabIter s = slab_slot(B, cnt);
  if (s.valid) {
    double v[3];
    load_vel<FORM>(P, s.i, v);
    double m = B.mass;
    if constexpr (EMB) {
      const uint32_t tg = P.tag[s.i];
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
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int q = 0; q < 10; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 10)
    atomicAdd(reinterpret_cast<unsigned long long*>(&tot[threadIdx.x]),
              (unsigned long long)red[threadIdx.x][0]);
  if (bad) atomicOr(&status[0], ERR_FIXED_RANGE);
}

// ------------------------------------------------------------ state I/O
// Row-major N x 3 doubles (tag order) -> internal form, placed in the slab of
// the tile of the particle's home cell. Pass 1 (PLACE == false) only counts
// per tile and checks the box; pass 2 writes.
template <int FORM, bool PLACE>
__global__ __launch_bounds__(256) void k_import(Particles P, Box B,
                                                const double* __restrict__ pos,
                                                const double* __restrict__ vel,
                                                uint32_t n, uint32_t tag0, uint32_t* cnt,
                                                uint32_t* bad_pos) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= n) return;
  double x[3], v[3];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d] = pos[3ull * t + d];
    v[d] = vel[3ull * t + d];
    bad |= !(x[d] >= 0.0 && x[d] < B.L[d]);
  }
  if (bad) {
    atomicOr(bad_pos, 1u);
    return;
  }
  Pos<FORM> r;
  const double w[3] = {v[0], v[1], v[2]};
  if constexpr (FORM == 0) {
    r.x[0] = x[0];
    r.x[1] = x[1];
    r.x[2] = x[2];
  } else {
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
      r.h[d] = hd;
      r.o[d] = o;
    }
  }
  int c[3];
  r.home3(B, c);
  const uint32_t T = tile_index(B, c);
  const uint32_t slot = atomicAdd(&cnt[T], 1u);
  if constexpr (PLACE) {
    if (slot < B.cap) {
      const size_t j = (size_t)T * B.cap + slot;
      store_vel<FORM>(P, j, w);
      P.tag[j] = tag0 + t;
      r.store(P, j);
    } else {
      atomicOr(bad_pos, 2u);
    }
  }
}

// Internal form -> row-major N x 3 doubles in tag order.
template <int FORM>
__global__ __launch_bounds__(256) void k_export(Particles P, Box B, const uint32_t* cnt,
                                                double* __restrict__ pos,
                                                double* __restrict__ vel) {
  const SlabIter s = slab_slot(B, cnt);
  if (!s.valid) return;
  const uint32_t t = P.tag[s.i];
  if constexpr (FORM == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pos[3ull * t + d] = P.x[d][s.i];
      vel[3ull * t + d] = P.v[d][s.i];
    }
  } else {
    int h[3];
    unpack_home(P.h[s.i], h[0], h[1], h[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pos[3ull * t + d] = (double)h[d] * B.a + (double)P.o[d][s.i];
      vel[3ull * t + d] = (double)P.vf[d][s.i];
    }
  }
}

// Copy the valid slots of every tile from slabs of capacity old_cap to slabs
// of capacity B.cap (B.cap >= old_cap); used when slabs are enlarged.
template <int FORM>
__global__ __launch_bounds__(256) void k_repack(Particles src, Particles dst, Box B,
                                                uint32_t old_cap, const uint32_t* cnt) {
  const uint32_t per = (old_cap + 255u) / 256u;
  const uint32_t T = blockIdx.x / per;
  const uint32_t k = (blockIdx.x % per) * 256u + threadIdx.x;
  if (T >= B.ntiles || k >= min(cnt[T], old_cap)) return;
  const size_t i = (size_t)T * old_cap + k, j = (size_t)T * B.cap + k;
  double v[3];
  load_vel<FORM>(src, i, v);
  store_vel<FORM>(dst, j, v);
  Pos<FORM> r;
  r.load(src, i);
  r.store(dst, j);
  dst.tag[j] = src.tag[i];
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
