// Kernels of the SRD step on gfx950 (wave64, 160 KB LDS per CU, 8 XCDs).
//
// Data layout in HBM. The box is cut into tiles of td[0] x td[1] x td[2]
// cells (4x4x2 to 8x8x4). Every tile owns a slab of `cap` particle slots in
// each of two buffers; the first cnt[T] slots of tile T hold its particles in
// no particular order. Within a slab the data is structure of arrays, one
// array per component, so a block reads and writes its tile as unit-stride
// streams:
//   FP64 form: three 16-byte words per particle, wa[S] = {x, y},
//              wb[S] = {z, v_x}, wc[S] = {v_y, v_z} (double), and tag[S];
//   FP32 form: two 16-byte words per particle, ra[S] = {home cell packed
//              10:10:10, float offset inside the home cell x, y, z} and
//              rb[S] = {float velocity x, y, z, tag}, so a lane moves a
//              particle with two vector loads or stores;
//   tag[S] uint32 particle identity (FP64 form; inside rb in the FP32 form);
//   S = ntiles * cap. A particle's cell inside its tile is not stored: the
//   collision recomputes it from the position and the step's shift.
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
  int tsh[3];          // cell -> tile coordinate: c >> tsh (log2(td); 31 if nt == 1)
  int nt[3];           // tiles per axis
  uint32_t lm[3];      // cell -> cell inside its tile: c & lm (td - 1, or all ones if nt == 1)
  uint32_t m_td0, m_td01;   // ceil(2^24 / td[0]), ceil(2^24 / (td[0] td[1]))
  double inv_nt0, inv_nt01; // 1 / nt[0], 1 / (nt[0] nt[1])
  uint32_t ntiles;     // tiles of this box
  uint32_t tile0;      // its first tile in the slab arrays
  uint32_t tag0;       // its first particle tag
  uint32_t cell0;      // its first cell in per-cell outputs
  uint32_t md_solute;  // 1: embedded particles are moved by an external MD integrator, not streamed
};

// Whether the MPCD stream moves particle `tag` (embedded particles are left to
// the MD integrator when the box couples solutes that way, sec. 3.6).
__device__ inline bool streamed(const Box& B, uint32_t tag) {
  return !(B.md_solute && tag - B.tag0 >= B.n_solvent);
}
// The same in a kernel that knows whether its tiles can hold embedded
// particles (without them every particle streams).
template <bool MAY_EMB>
__device__ inline bool streamed_in(const Box& B, uint32_t tag) {
  if constexpr (MAY_EMB) return streamed(B, tag);
  return true;
}

// Several independent boxes share one set of slabs: box b owns the tiles
// [tile0, tile0 + ntiles), its particles carry the tags [tag0, tag0 + n).
struct Slabs {
  const Box* boxes;          // per box, device memory
  const uint32_t* tile_box;  // tile -> box
  uint32_t ntiles;           // tiles of all boxes
  uint32_t cap;              // slots per tile
};

// Grid shift of one box for one step (sec. 2), in FP64 and rounded to FP32.
struct ShiftEntry {
  double s[3];
  float s32[3];
  float pad;
};

struct Particles {
  double2* wa;   // FP64 form: {x, y}, {z, v_x}, {v_y, v_z} in three 16-byte words
  double2* wb;
  double2* wc;
  uint32_t* tag; // FP64 form: tag
  uint4* ra;     // FP32 form: {home cell packed 10:10:10, offset x, y, z (FP32 bits)}
  uint4* rb;     // FP32 form: {velocity x, y, z (FP32 bits), tag}
};

template <int FORM>
struct VelT {
  using T = double;
};
template <>
struct VelT<1> {
  using T = float;
};

// Slab element access. Inside one tile a 32-bit index k < cap addresses an
// element as a 32-bit byte offset from the tile's base pointer, which is
// uniform over the block (kept in scalar registers); a 64-bit index j is a
// position in the whole slab array (scatter to another tile, elementwise
// kernels). The tile capacity is below 2^28, so k * sizeof(T) fits 32 bits.
// Slab data is streamed: read once and written once per step, far more of
// it than the caches hold. Loads of the FP32 form's 16-byte particle words
// are nontemporal (measured faster); stores stay ordinary, because a block's
// scattered partial-line stores rely on write combining in L2, and the FP64
// form's loads measured slower with the hint.
template <class T>
struct NtType {
  using type = T;
};
template <class T>
struct NtLoad {
  static constexpr bool value = false;
};
template <>
struct NtLoad<uint4> {
  static constexpr bool value = true;
};
template <>
struct NtType<uint4> {
  typedef unsigned int type __attribute__((ext_vector_type(4)));
};
template <>
struct NtType<double2> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <class T>
__device__ inline T nt_load(const T* p) {
  using V = typename NtType<T>::type;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  T out;
  __builtin_memcpy(&out, &v, sizeof(T));
  return out;
}
template <class T>
__device__ inline void nt_store(T* p, T x) {
  using V = typename NtType<T>::type;
  V v;
  __builtin_memcpy(&v, &x, sizeof(T));
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

template <class T>
__device__ inline T ld_at(const T* p) {
  if constexpr (NtLoad<T>::value) return nt_load(p);
  else return *p;
}
template <class T>
__device__ inline T ld(const T* base, uint32_t k) {
  return ld_at(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                          (uint32_t)(k * (uint32_t)sizeof(T))));
}
template <class T>
__device__ inline void st(T* base, uint32_t k, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(k * (uint32_t)sizeof(T))) = v;
}
template <class T>
__device__ inline T ld(const T* base, size_t j) {
  return ld_at(base + j);
}
template <class T>
__device__ inline void st(T* base, size_t j, T v) {
  base[j] = v;
}

// The arrays of one form advanced to slot `off` (the first slot of a tile).
template <int FORM>
__device__ inline Particles tile_view(const Particles& P, size_t off) {
  Particles Q = P;
  if constexpr (FORM == 0) {
    Q.wa = P.wa + off;
    Q.wb = P.wb + off;
    Q.wc = P.wc + off;
    Q.tag = P.tag + off;
  } else {
    Q.ra = P.ra + off;
    Q.rb = P.rb + off;
  }
  return Q;
}

// Blocks are handed to the 8 XCDs round-robin; remapping makes XCD k work on
// one contiguous range of tiles, so neighbouring tiles share its L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u;
  const uint32_t x = b & 7u, i = b >> 3;
  return x < r ? x * (q + 1u) + i : r * (q + 1u) + (x - r) * q + i;
}

// Division without the integer divide sequence. l / d for l < 256 and
// d <= 64 (tile sizes are at most 8 cells per axis): with m = ceil(2^24 / d),
// floor(l m / 2^24) is exact whenever l d < 2^24.
__device__ inline uint32_t div_small(uint32_t l, uint32_t m24) { return (l * m24) >> 24; }

// T / d for any 32-bit T: an FP64 estimate, corrected by one step.
__device__ inline uint32_t div_tile(uint32_t T, uint32_t d, double inv) {
  uint32_t q = (uint32_t)((double)T * inv);
  if (q * d > T) --q;
  else if ((q + 1u) * d <= T) ++q;
  return q;
}

// Tile coordinates of tile T (x fastest).
__device__ inline void tile_coords(const Box& B, uint32_t T, int t3[3]) {
  const uint32_t n0 = (uint32_t)B.nt[0], n1 = (uint32_t)B.nt[1];
  const uint32_t a = div_tile(T, n0, B.inv_nt0);
  const uint32_t z = div_tile(T, n0 * n1, B.inv_nt01);
  t3[0] = (int)(T - a * n0);
  t3[1] = (int)(a - z * n1);
  t3[2] = (int)z;
}

// Coordinates of local cell l inside a tile (x fastest).
__device__ inline void local_coords(const Box& B, uint32_t l, uint32_t l3[3]) {
  const uint32_t a = div_small(l, B.m_td0);
  const uint32_t z = div_small(l, B.m_td01);
  l3[0] = l - __umul24(a, (uint32_t)B.td[0]);
  l3[1] = a - __umul24(z, (uint32_t)B.td[1]);
  l3[2] = z;
}

// Tile coordinate of cell coordinate c (0 <= c < n < 2^10) along axis d.
__device__ inline int tile_coord(int c, const Box& B, int d) {
  return c >> B.tsh[d];
}

// Index products of cell and tile coordinates: every factor is below 2^24
// (at most 1023 cells per axis), so the 24-bit multiply-add gives the exact
// 32-bit result at full rate.
__device__ inline uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
  return __umul24(a, b) + c;
}

// Velocity and tag of a particle. Both forms keep a particle in 16-byte
// words, so a lane moves it with few vector loads and stores.
template <int FORM, class I>
__device__ inline void load_vt(const Particles& P, I i, typename VelT<FORM>::T v[3], uint32_t& tag) {
  if constexpr (FORM == 0) {
    const double2 b = ld(P.wb, i), c = ld(P.wc, i);
    v[0] = b.y;
    v[1] = c.x;
    v[2] = c.y;
    tag = ld(P.tag, i);
  } else {
    const uint4 b = ld(P.rb, i);
    v[0] = __uint_as_float(b.x);
    v[1] = __uint_as_float(b.y);
    v[2] = __uint_as_float(b.z);
    tag = b.w;
  }
}

template <int FORM, class I>
__device__ inline void load_vel(const Particles& P, I i, typename VelT<FORM>::T v[3]) {
  uint32_t tag;
  load_vt<FORM>(P, i, v, tag);
}

template <int FORM, class I>
__device__ inline uint32_t load_tag(const Particles& P, I i) {
  if constexpr (FORM == 0) return ld(P.tag, i);
  else return ld(reinterpret_cast<const uint32_t*>(P.rb), (I)(4 * i + 3));
}



// Position of one particle in registers: stream (eq. 1) and bin (sec. 3.4).
template <int FORM>
struct Pos;
template <>
struct Pos<0> {
  double x[3];
  template <class I>
  __device__ void load(const Particles& P, I i) {
    const double2 a = ld(P.wa, i);
    x[0] = a.x;
    x[1] = a.y;
    x[2] = ld(P.wb, i).x;
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
  uint32_t hp;  // home cell, packed 10:10:10
  float o[3];
  template <class I>
  __device__ void load(const Particles& P, I i) {
    const uint4 a = ld(P.ra, i);
    hp = a.x;
    o[0] = __uint_as_float(a.y);
    o[1] = __uint_as_float(a.z);
    o[2] = __uint_as_float(a.w);
  }
  __device__ void stream(const Box& B, const float v[3], uint32_t&) {
    int h[3];
    unpack_home(hp, h[0], h[1], h[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) stream_axis32(o[d], h[d], v[d], B.dt32, B.a32, B.inv_a32, B.n[d]);
    hp = pack_home(h[0], h[1], h[2]);
  }
  __device__ void cell3(const Box& B, const double*, const float s32[3], int c[3]) const {
    int h[3];
    unpack_home(hp, h[0], h[1], h[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = bin_axis32(o[d], h[d], s32[d], B.inv_a32, B.n[d]);
  }
  __device__ void home3(const Box&, int c[3]) const { unpack_home(hp, c[0], c[1], c[2]); }
};

// Position records staged in LDS (16 bytes per particle): the FP32 form's
// whole position word {home cell, offset x, y, z}; the FP64 form's {x, y},
// whose z travels in the velocity word and stays in a register.
__device__ inline void pos_from_lds(const uint4& a, double, Pos<1>& r) {
  r.hp = a.x;
  r.o[0] = __uint_as_float(a.y);
  r.o[1] = __uint_as_float(a.z);
  r.o[2] = __uint_as_float(a.w);
}
__device__ inline void pos_from_lds(const uint4& a, double z, Pos<0>& r) {
  r.x[0] = __hiloint2double((int)a.y, (int)a.x);
  r.x[1] = __hiloint2double((int)a.w, (int)a.z);
  r.x[2] = z;
}
__device__ inline uint4 pos_to_lds(const Pos<1>& r) {
  return make_uint4(r.hp, __float_as_uint(r.o[0]), __float_as_uint(r.o[1]), __float_as_uint(r.o[2]));
}
__device__ inline uint4 pos_to_lds(const Pos<0>& r) {
  return make_uint4((uint32_t)__double2loint(r.x[0]), (uint32_t)__double2hiint(r.x[0]),
                    (uint32_t)__double2loint(r.x[1]), (uint32_t)__double2hiint(r.x[1]));
}

// Issue the load of the 16-byte position record of slot k of a tile straight
// into LDS (global_load_lds_dwordx4): lane l of the wave writes
// lds_wave + l. Completion is awaited with s_waitcnt before the LDS is read.
// The FP32 form's records are read nontemporally, as its other loads are.
template <int FORM>
__device__ inline void stage_pos(const Particles& P, uint32_t k, uint4* lds_wave) {
  const char* base = FORM == 0 ? reinterpret_cast<const char*>(P.wa) : reinterpret_cast<const char*>(P.ra);
  constexpr int NT = FORM == 1 ? 2 : 0;  // cache policy: the nt bit
  __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(base + (uint32_t)(k * 16u)),
                                   (__attribute__((address_space(3))) void*)(lds_wave), 16, 0, NT);
}

// Velocity and tag of slot k, and the FP64 form's z (in the same word).
template <int FORM>
__device__ inline void load_vt_z(const Particles& P, uint32_t k, typename VelT<FORM>::T v[3],
                                 uint32_t& tag, double& z) {
  if constexpr (FORM == 0) {
    const double2 b = ld(P.wb, k), c = ld(P.wc, k);
    z = b.x;
    v[0] = b.y;
    v[1] = c.x;
    v[2] = c.y;
    tag = ld(P.tag, k);
  } else {
    load_vt<FORM>(P, k, v, tag);
    z = 0.0;
  }
}

// A whole particle: position, velocity and tag.
template <int FORM, class I>
__device__ inline void load_part(const Particles& P, I i, Pos<FORM>& r, typename VelT<FORM>::T v[3],
                                 uint32_t& tag) {
  if constexpr (FORM == 0) {
    const double2 a = ld(P.wa, i), b = ld(P.wb, i), c = ld(P.wc, i);
    r.x[0] = a.x;
    r.x[1] = a.y;
    r.x[2] = b.x;
    v[0] = b.y;
    v[1] = c.x;
    v[2] = c.y;
    tag = ld(P.tag, i);
  } else {
    r.load(P, i);
    load_vt<FORM>(P, i, v, tag);
  }
}

template <int FORM, class I>
__device__ inline void store_part(const Particles& P, I j, const Pos<FORM>& r,
                                  const typename VelT<FORM>::T w[3], uint32_t tag) {
  if constexpr (FORM == 0) {
    st(P.wa, j, make_double2(r.x[0], r.x[1]));
    st(P.wb, j, make_double2(r.x[2], w[0]));
    st(P.wc, j, make_double2(w[1], w[2]));
    st(P.tag, j, tag);
  } else {
    st(P.ra, j, make_uint4(r.hp, __float_as_uint(r.o[0]), __float_as_uint(r.o[1]), __float_as_uint(r.o[2])));
    st(P.rb, j, make_uint4(__float_as_uint(w[0]), __float_as_uint(w[1]), __float_as_uint(w[2]), tag));
  }
}

// The velocity-bearing words of record j only (position words unchanged).
template <int FORM, class I>
__device__ inline void store_vel(const Particles& P, I j, const Pos<FORM>& r,
                                 const typename VelT<FORM>::T w[3], uint32_t tag) {
  if constexpr (FORM == 0) {
    st(P.wb, j, make_double2(r.x[2], w[0]));
    st(P.wc, j, make_double2(w[1], w[2]));
  } else {
    st(P.rb, j, make_uint4(__float_as_uint(w[0]), __float_as_uint(w[1]), __float_as_uint(w[2]), tag));
  }
}

__device__ inline uint32_t cell_index(const Box& B, const int c[3]) {
  return mad24((uint32_t)B.n[0], mad24((uint32_t)B.n[1], (uint32_t)c[2], (uint32_t)c[1]), (uint32_t)c[0]);
}

__device__ inline uint32_t tile_index(const Box& B, const int c[3]) {
  const int tx = tile_coord(c[0], B, 0), ty = tile_coord(c[1], B, 1), tz = tile_coord(c[2], B, 2);
  return mad24((uint32_t)B.nt[0], mad24((uint32_t)B.nt[1], (uint32_t)tz, (uint32_t)ty), (uint32_t)tx);
}

// ------------------------------------------------------- scatter helpers
// Tile at offset (bin % 3 - 1, bin / 3 % 3 - 1, bin / 9 - 1) from tile t,
// periodic.
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

// Cell c's index inside its tile (x fastest).
__device__ inline uint32_t local_cell(const Box& B, const int c[3]) {
  return mad24((uint32_t)B.td[0],
               mad24((uint32_t)B.td[1], (uint32_t)c[2] & B.lm[2], (uint32_t)c[1] & B.lm[1]),
               (uint32_t)c[0] & B.lm[0]);
}

// Where a particle in cell c goes from tile t: its bin 0..26 among the 27
// neighbour tiles, or 27 for any other tile; and its cell inside the
// destination tile. Per axis the tile offset diff (in (-nt, nt)) is taken
// periodically into [-1, 1] where it names a neighbour: down by nt if
// above 1, then up by nt if below -1 (with nt == 2 the tile at +1 is also
// the one at -1, and either bin names it).
__device__ inline uint32_t dest_bin(const Box& B, const int t[3], const int c[3], uint32_t& lcell) {
  uint32_t bin = 0, far = 0;
  constexpr uint32_t mul[3] = {1u, 3u, 9u};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int nt = B.nt[d];
    int diff = tile_coord(c[d], B, d) - t[d];
    diff -= diff > 1 ? nt : 0;
    diff += diff < -1 ? nt : 0;
    const uint32_t o = (uint32_t)(diff + 1);  // 0, 1, 2 for a neighbour
    far = max(far, o);
    bin += o * mul[d];
  }
  lcell = local_cell(B, c);
  return far > 2u ? 27u : bin;
}

// ------------------------------------------------------------ tile kernel
enum { MODE_BIN = 0, MODE_COLLIDE = 1, MODE_COLLIDE_SCATTER = 2, MODE_DIAG = 3 };

constexpr int TT = 256;         // threads per tile block
constexpr uint32_t LC_PEND = 0x100u;  // in a particle's local cell: its cell's draw is pending
// particles per thread held in registers (beyond TT * TQ a tile's particles
// are re-read from memory): 3 for 64-cell tiles (up to 768 particles, used
// at densities 7..11), 4 otherwise
constexpr int tq_for(int cpt) { return cpt == 64 ? 3 : 4; }

struct TileArgs {
  Particles in, out;
  Slabs S;
  const uint32_t* cnt_in;   // occupancy of the input slabs
  uint32_t* cnt_out;        // occupancy of the output slabs (scatter modes)
  uint32_t* cnt_clear;      // cleared for this tile (scatter modes)
  const double* emb_mass;
  uint32_t step;            // counter of the collision
  const ShiftEntry* sh;     // per box: shift binning the input (collide) or output (bin)
  const ShiftEntry* shn;    // per box: shift of the next step (collide + scatter)
  uint32_t* status;
  uint32_t seq;             // launch sequence number within one API call
  double* d_mass;           // per-cell outputs of MODE_DIAG (global cell index)
  double* d_mom;
  double* d_ek;
  double* d_axis;
  double* d_xi;
  uint32_t* eslot_out;      // slot of each embedded particle in the output
                            // buffer (null without embedded particles)
  uint32_t one_box;         // 1: a single box (every tile's box is 0; the
                            // tile -> box table need not be read)
};

// Record the slot j of an embedded particle (tag) in the index of the buffer
// it was written to; solvent particles are not indexed.
__device__ inline void note_slot(uint32_t* eslot, const Box& B, uint32_t tag, size_t j) {
  const uint32_t i = tag - B.tag0;
  if (i >= B.n_solvent) eslot[i - B.n_solvent] = (uint32_t)j;
}

// Fixed-point accumulator rows of one cell sum: the FP64 form keeps two limbs
// (fx_split), the FP32 form one (fx1_split).
template <int FORM>
struct Acc {
  static constexpr int NL = FORM == 0 ? 2 : 1;
  __device__ static void add(unsigned long long* row0, unsigned long long* row1, double x, bool& bad) {
    if constexpr (NL == 2) {
      long long hi, lo;
      fx_split(x, hi, lo, bad);
      atomicAdd(row0, (unsigned long long)hi);
      atomicAdd(row1, (unsigned long long)lo);
    } else {
      atomicAdd(row0, (unsigned long long)fx1_split(x, bad));
    }
  }
  __device__ static double value(unsigned long long a0, unsigned long long a1) {
    if constexpr (NL == 2) {
      Fx f;
      f.hi = (long long)a0;
      f.lo = (long long)a1;
      return fx_value(f);
    } else {
      return fx1_value((long long)a0);
    }
  }
};

// AT kick of particle i of its box in the form's precision (FP64 form:
// at_kick; FP32 form: at_kick32, returned exactly in FP64).
template <int FORM>
__device__ inline void at_kick_form(uint32_t i, uint32_t step, uint32_t k0, uint32_t k1,
                                    double scale, double dv[3]) {
  if constexpr (FORM == 0) {
    at_kick(i, step, k0, k1, scale, dv);
  } else {
    float f[3];
    at_kick32(i, step, k0, k1, (float)scale, f);
#pragma unroll
    for (int d = 0; d < 3; ++d) dv[d] = (double)f[d];
  }
}

// AT kick of a particle beyond the register-resident part of its tile. Kept
// out of line: drawn inline there, its Box-Muller chain would be scheduled
// around the live register-resident particles and raise every wave's
// register count (FP32 form with FP64 kicks: 88 -> 74 VGPRs), although only
// crowded tiles take that path.
template <int FORM>
__device__ __noinline__ void at_kick_tail(uint32_t i, uint32_t step, uint32_t k0, uint32_t k1,
                                          double scale, double dv[3]) {
  at_kick_form<FORM>(i, step, k0, k1, scale, dv);
}

// Maxwell-Boltzmann draw of a cell with nc >= 2 particles (sec. 3.6):
// E_hat ~ Gamma(3 (nc - 1) / 2, kT) by Marsaglia and Tsang's sampler.
// The numbers of an attempt depend on (cell, step, attempt) only, so those of
// attempts 0 and 1 are drawn before N_c is known: the normal g and lu =
// log U, or -inf where the squeeze (which needs no N_c either) accepts.
// gamma_first2 decides these two attempts as gamma_mt would; it returns -1
// when both are rejected (about one cell in 10^3), and gamma_mt from attempt
// 2 finishes the draw.
constexpr int GPRE = 2;  // attempts drawn ahead

__device__ inline double gamma_first2(uint32_t nc, const double g[GPRE], const double lu[GPRE],
                                      double theta) {
  const double k = 1.5 * (double)(nc - 1u);
  const double d = k - 1.0 / 3.0;
  const double c = 1.0 / sqrt(9.0 * d);
#pragma unroll
  for (int j = 0; j < GPRE; ++j) {
    const double t = 1.0 + c * g[j];
    const double V = t * t * t;
    if (t > 0.0 && (lu[j] == -INFINITY || gamma_full_log(g[j], V, lu[j], d))) return d * V * theta;
  }
  return -1.0;
}

__device__ inline double gamma_finish(uint32_t nc, uint32_t cell, uint32_t step, const Box& B,
                                      uint32_t& err) {
  bool cap = false;
  const double e = gamma_mt(1.5 * (double)(nc - 1u), cell, step, B.k0, B.k1, B.kT, cap, (uint32_t)GPRE);
  if (cap) err |= ERR_GAMMA_CAP;
  return e;
}

// One block per tile. In the per-cell phases thread l < CPT works for cell
// l: it draws the axis (and the numbers of the first attempts of the
// thermostat's Gamma draw) while the tile's particles load, and once the cell
// sums are in, decides the Gamma draw and forms u, xi and the rotation. The
// particles of the rare cells whose draw needs a third attempt are left out
// of the main pass: once it is done and the registers holding the tile are
// free, their cell threads finish the draw, and those particles are read
// again from the input slab, rotated and scattered one by one.
// ATR: the Andersen-thermostat rule (eq. 4) instead of the rotation; every
// particle draws a random velocity dv in the gather, the cell sums gain
// sum m dv, and the update is v <- (u + dv) - sum m dv / M.
// Register targets (waves per SIMD) of the FP32 rotation kernels, measured:
// 64-cell tiles eight (64 VGPRs, with the LDS of a block under 20 KB so that
// eight blocks fit a CU: the thermostatted step ~1.4 % faster than at seven,
// though a few dwords spill; with embedded particles the compiler cannot
// meet eight and seven is kept), thermostatted 128-cell tiles seven (72
// VGPRs, a few spilled dwords; ~1 % faster than six at densities 4-7, six
// ~3 % faster than the compiler's own choice); under the AT rule 64-cell
// tiles eight (single-precision kicks, kept in LDS as FP32: 60-64 VGPRs and
// 16 KB of LDS per block; 153 against 160 us at six).
template <int FORM, int CPT, int MODE, bool STREAM_IN, bool THERMO, bool EMB, bool ATR>
constexpr int tile_waves_per_eu() {
  if (FORM != MPCD_FP32) return 1;
  if (ATR) return CPT == 64 ? 8 : 1;  // AT rule, 64-cell tiles: eight
  if (CPT == 64) return EMB ? 7 : 8;
  if (CPT == 128 && THERMO) return 7;
  return 1;
}

template <int FORM, int CPT, int MODE, bool STREAM_IN, bool THERMO, bool EMB, bool ATR>
__global__ __launch_bounds__(TT) __attribute__((amdgpu_waves_per_eu(
    tile_waves_per_eu<FORM, CPT, MODE, STREAM_IN, THERMO, EMB, ATR>()))) void k_tile(TileArgs A) {
  using VT = typename VelT<FORM>::T;
  using AC = Acc<FORM>;
  constexpr bool COLL = MODE != MODE_BIN;
  constexpr bool SCAT = MODE == MODE_BIN || MODE == MODE_COLLIDE_SCATTER;
  constexpr bool EK = THERMO || MODE == MODE_DIAG;
  constexpr bool AT = ATR && COLL && MODE != MODE_DIAG;
  // binning launches share one instantiation with and without embedded
  // particles: they check each particle's tag
  constexpr bool MAY_EMB = EMB || MODE == MODE_BIN;
  // 64-cell step kernels of the SRD rule keep the register-resident
  // particles' position records in LDS (loaded there directly) instead of
  // registers: positions are needed only after the rotation, and the
  // registers go to occupancy (the AT rule's kicks already fill its LDS)
  constexpr bool LPOS = (MODE == MODE_COLLIDE || MODE == MODE_COLLIDE_SCATTER) && CPT == 64 && !ATR;
  constexpr int NL = AC::NL;
  constexpr int TQ = tq_for(CPT);
  constexpr int TREG = TT * TQ;
  constexpr int RP = 0;                       // momentum rows: RP + NL * axis
  constexpr int RQ = 3 * NL;                  // AT: sum m dv rows, RQ + NL * axis
  constexpr int RE = AT ? RQ + 3 * NL : RQ;   // relative kinetic energy
  constexpr int RM = EK ? RE + NL : RE;       // mass (embedded particles)
  constexpr int NROW = COLL ? RM + (EMB ? NL : 0) : 1;
  constexpr int CC = COLL ? CPT : 1;
  static_assert(CPT <= 256 && (CPT & (CPT - 1)) == 0, "cells per tile: a power of two <= 256");
  __shared__ unsigned long long s_acc[NROW][CC];
  __shared__ uint32_t s_cnt[CC];
  __shared__ double s_u[3][CC];
  __shared__ double s_ax[3][CC];  // per cell: the rotation axis (SRD) or the mean kick (AT)

  // thermostat: attempts 0 and 1 of the cell's Gamma draw, normal g and log U
  // (-inf where the squeeze accepts), drawn before N_c is known; cells whose
  // draw is not decided by them (pending) and whether the block has any
  __shared__ double s_gam[THERMO ? 2 * GPRE : 2][THERMO ? CC : 1];
  // the drawn energy and xi reuse the rows of the first two attempts: a cell's
  // thread reads its column before it writes Ehat there, and xi is written
  // barriers after the last read
  auto& s_ehat = s_gam[0];
  auto& s_xi = s_gam[1];
  __shared__ uint32_t s_pend[THERMO ? CC : 1];
  __shared__ uint32_t s_anyp;
  __shared__ uint32_t s_bincnt[27];
  __shared__ uint32_t s_base[27];
  __shared__ uint32_t s_btile[27];
  __shared__ uint32_t s_quit;

  const uint32_t tid = threadIdx.x;
  const uint32_t T = xcd_remap(blockIdx.x, gridDim.x);  // tile, all boxes
  const uint32_t bx = A.one_box ? 0u : A.S.tile_box[T];
  const Box B = A.S.boxes[bx];  // a copy: loaded once, not re-read after stores
  const uint32_t cap = A.S.cap;
  int t3[3];
  tile_coords(B, T - B.tile0, t3);
  // this box's shifts, copied once: binning the input (or the output in
  // MODE_BIN), and binning the next step's input (MODE_COLLIDE_SCATTER)
  const ShiftEntry sh0 = A.sh[bx];
  ShiftEntry sh1{};
  if constexpr (MODE == MODE_COLLIDE_SCATTER) sh1 = A.shn[bx];
  const double* sd = sh0.s;
  const float* sd32 = sh0.s32;

  // The status word, the occupancy and then the tile's particles are loaded
  // before the first barrier, so their latencies overlap. A block quits
  // after it if an earlier launch of this call overflowed a slab (launches
  // of the failing one itself run to the end, so its counts are complete).
  if (tid == 0) {
    s_quit = (A.status[1] != 0u && A.status[2] < A.seq) ? 1u : 0u;
    if constexpr (THERMO) s_anyp = 0u;
  }
  const uint32_t cnt = min(A.cnt_in[T], cap);
  const uint32_t nreg = min(cnt, (uint32_t)TREG);
  const size_t tbase = (size_t)T * cap;
  const Particles In = tile_view<FORM>(A.in, tbase);
  if (tid < 27u) {
    s_bincnt[tid] = 0u;
    if constexpr (SCAT) s_btile[tid] = B.tile0 + bin_tile(B, t3, tid);
  }
  if constexpr (COLL) {
    for (uint32_t t = tid; t < (uint32_t)(NROW * CC); t += TT) (&s_acc[0][0])[t] = 0ull;
    if (tid < (uint32_t)CC) s_cnt[tid] = 0u;
  }

  uint32_t err = 0;
  bool bad = false;

  auto mass_of = [&](uint32_t tag) -> double {
    if constexpr (EMB) {
      const uint32_t i = tag - B.tag0;
      return i >= B.n_solvent ? A.emb_mass[i - B.n_solvent] : B.mass;
    } else {
      return B.mass;
    }
  };
  // global index of local cell l, and whether the cell exists (the last
  // tile along an axis may be partial)
  auto cell_of = [&](uint32_t l, bool& ok) -> uint32_t {
    uint32_t l3[3];
    local_coords(B, l, l3);
    const int g[3] = {t3[0] * B.td[0] + (int)l3[0], t3[1] * B.td[1] + (int)l3[1], t3[2] * B.td[2] + (int)l3[2]};
    ok = l < (uint32_t)CPT && l3[2] < (uint32_t)B.td[2] && g[0] < B.n[0] && g[1] < B.n[1] &&
         g[2] < B.n[2];
    return ok ? cell_index(B, g) : 0u;
  };
  // a particle's cell inside this tile: its cell under this step's shift,
  // which the launch that placed it in this slab computed too (recomputed
  // from the position rather than stored: a byte per particle written and
  // read again cost more than the arithmetic)
  auto lc_from = [&](const Pos<FORM>& rr) -> uint32_t {
    int c[3];
    rr.cell3(B, sd, sd32, c);
    return local_cell(B, c) & (uint32_t)(CPT - 1);
  };
  auto lc_at = [&](uint32_t k) -> uint32_t {
    Pos<FORM> rr;
    typename VelT<FORM>::T vv[3];
    uint32_t t;
    load_part<FORM>(In, k, rr, vv, t);
    return lc_from(rr);
  };

  // The per-cell draws need only (cell, step). The block's threads form
  // TT / CPT groups of CPT lanes, lane l of each group working for cell l:
  // group 0 (the cell threads) draws the axis, and the numbers of each of
  // the first attempts of the thermostat draw come from a group of their
  // own where the tile leaves one (64-cell tiles: attempt j on group 1 + j),
  // so the chains run side by side on different waves. They are drawn while
  // the tile's count is in flight, before the gather (drawn after the gather
  // is issued, they would be scheduled against the registers the loads
  // fill), and wait in LDS.
  constexpr uint32_t NG = TT / CPT;                 // lane groups
  const uint32_t grp = tid / (uint32_t)CPT, gl = tid & (uint32_t)(CPT - 1);
  constexpr uint32_t DG = NG > 1 ? 1u : 0u;         // the group that decides the draws
  const bool cthr = COLL && grp == 0u;
  bool cok = false;
  const uint32_t gcell = cthr ? cell_of(tid, cok) : 0u;
  const bool gthr = THERMO && COLL && grp == DG;
  if constexpr (COLL) {
    if (cthr && !AT) {
      double n[3] = {0.0, 0.0, 0.0};
      if (cok) cell_axis(gcell, A.step, B.k0, B.k1, n);
      s_ax[0][tid] = n[0];
      s_ax[1][tid] = n[1];
      s_ax[2][tid] = n[2];
    }
    if constexpr (THERMO) {
#pragma unroll
      for (int j = 0; j < GPRE; ++j) {
        if (grp == min(DG + (uint32_t)j, NG - 1u)) {
          bool ok;
          const uint32_t c = cell_of(gl, ok);
          double g = 0.0, lu = -INFINITY;
          if (ok) {
            double u2;
            gamma_numbers(c, A.step, (uint32_t)j, B.k0, B.k1, g, u2);
            if (!gamma_squeeze(g, u2)) lu = log(u2);
          }
          s_gam[2 * j][gl] = g;
          s_gam[2 * j + 1][gl] = lu;
        }
      }
    }
  }

  // ---- gather this tile's particles (register-resident part)
  VT v[TQ][3];
  uint32_t tg[TQ];
  uint32_t lcs[TQ];
  Pos<FORM> r[TQ];                             // positions in registers (not with LPOS)
  __shared__ uint4 s_pos[LPOS ? TREG : 1];     // LPOS: position records, slot k at k
  double zq[LPOS && FORM == 0 ? TQ : 1];       // LPOS, FP64 form: z of each position
  // AT rule: each register-resident particle's kick, drawn once and used by
  // the cell sums and the update, waits in LDS in the form's precision (in
  // registers it would hold 3 to 6 VGPRs per particle slot through the whole
  // kernel and cut occupancy)
  __shared__ VT s_dv[AT ? 3 : 1][AT ? TREG : 1];
  auto kick = [&](uint32_t tag, double m, double out[3]) {
    at_kick_form<FORM>(tag - B.tag0, A.step, B.k0, B.k1, sqrt(B.kT / m), out);
  };
#pragma unroll
  for (int q = 0; q < TQ; ++q) {
    const uint32_t k = tid + (uint32_t)(q * TT);
    lcs[q] = 0u;
    tg[q] = 0u;
    if (k < nreg) {
      if constexpr (LPOS) {
        stage_pos<FORM>(In, k, &s_pos[(uint32_t)(q * TT) + (tid & ~63u)]);
        double z;
        load_vt_z<FORM>(In, k, v[q], tg[q], z);
        if constexpr (FORM == 0) zq[q] = z;
      } else {
        load_part<FORM>(In, k, r[q], v[q], tg[q]);
      }
      if constexpr (COLL && !LPOS) lcs[q] = lc_from(r[q]);
    }
  }
  if constexpr (LPOS) {
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const uint32_t k = tid + (uint32_t)(q * TT);
      if (k < nreg) {
        Pos<FORM> rr;
        pos_from_lds(s_pos[k], FORM == 0 ? zq[q] : 0.0, rr);
        lcs[q] = lc_from(rr);
      }
    }
  }
  if constexpr (AT) {
#pragma unroll
    for (int q = 0; q < TQ; ++q)
      if (tid + (uint32_t)(q * TT) < nreg) {
        double kv[3];
        kick(tg[q], mass_of(tg[q]), kv);
#pragma unroll
        for (int d = 0; d < 3; ++d) s_dv[d][tid + (uint32_t)(q * TT)] = kv[d];
      }
  }

  __syncthreads();
  if (s_quit) return;
  if (SCAT && tid == 0 && A.cnt_clear) A.cnt_clear[T] = 0u;

  // ---- scatter: bin for the destination shift, reserve slots, write
  auto overflow = [&]() {
    atomicMax(&A.status[1], 1u);
    atomicMin(&A.status[2], A.seq);
  };
  auto put = [&](size_t j, const VT w[3], uint32_t tag, const Pos<FORM>& rr, uint32_t lcell) {
    store_part<FORM>(A.out, j, rr, w, tag);
    (void)lcell;
    if (A.eslot_out) note_slot(A.eslot_out, B, tag, j);
  };
  auto scatter = [&](const double* sd, const float* sd32, const VT (*w)[3]) {
    // per particle: local cell in the destination (bits 0-7), bin (8-12),
    // rank within the bin (13-31)
    uint32_t info[TQ];
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const uint32_t k = tid + (uint32_t)(q * TT);
      info[q] = 0u;
      if (k < nreg && !(lcs[q] & LC_PEND)) {
        int c[3];
        r[q].cell3(B, sd, sd32, c);
        uint32_t lcell;
        const uint32_t b = dest_bin(B, t3, c, lcell);
        const uint32_t rank = b < 27u ? atomicAdd(&s_bincnt[b], 1u) : 0u;
        info[q] = lcell | (b << 8) | (rank << 13);
      }
    }
    __syncthreads();
    if (tid < 27u && s_bincnt[tid] > 0u) s_base[tid] = atomicAdd(&A.cnt_out[s_btile[tid]], s_bincnt[tid]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
      const uint32_t k = tid + (uint32_t)(q * TT);
      if (k < nreg && !(lcs[q] & LC_PEND)) {
        const uint32_t b = (info[q] >> 8) & 31u;
        uint32_t dt, slot;
        if (b < 27u) {
          dt = s_btile[b];
          slot = s_base[b] + (info[q] >> 13);
        } else {
          int c[3];
          r[q].cell3(B, sd, sd32, c);
          dt = B.tile0 + tile_index(B, c);
          slot = atomicAdd(&A.cnt_out[dt], 1u);
        }
        if (slot < cap) put((size_t)dt * cap + slot, w[q], tg[q], r[q], info[q] & 255u);
        else overflow();
      }
    }
  };
  // particles beyond the register-resident part: one global atomic each
  auto scatter_one = [&](const Pos<FORM>& rr, const double* sd, const float* sd32, const VT w[3],
                         uint32_t tag) {
    int c[3];
    rr.cell3(B, sd, sd32, c);
    uint32_t lcell;
    (void)dest_bin(B, t3, c, lcell);
    const uint32_t dt = B.tile0 + tile_index(B, c);
    const uint32_t slot = atomicAdd(&A.cnt_out[dt], 1u);
    if (slot < cap) put((size_t)dt * cap + slot, w, tag, rr, lcell);
    else overflow();
  };

  if constexpr (MODE == MODE_BIN) {
    if constexpr (STREAM_IN) {
#pragma unroll
      for (int q = 0; q < TQ; ++q)
        if (tid + (uint32_t)(q * TT) < nreg && streamed_in<MAY_EMB>(B, tg[q])) r[q].stream(B, v[q], err);
    }
    scatter(sd, sd32, v);
    for (uint32_t k = TREG + tid; k < cnt; k += TT) {
      VT vv[3];
      uint32_t tag;
      Pos<FORM> rr;
      load_part<FORM>(In, k, rr, vv, tag);
      if (STREAM_IN && streamed_in<MAY_EMB>(B, tag)) rr.stream(B, vv, err);
      scatter_one(rr, sd, sd32, vv, tag);
    }
  } else {
    // ---- cell sums: count, momentum (and mass) in exact fixed point
    auto sum_mom = [&](uint32_t lc, const VT vv[3], double m, const double* kv) {
      atomicAdd(&s_cnt[lc], 1u);
#pragma unroll
      for (int d = 0; d < 3; ++d)
        AC::add(&s_acc[RP + NL * d][lc], &s_acc[RP + NL * d + NL - 1][lc], m * (double)vv[d], bad);
      if constexpr (AT) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          AC::add(&s_acc[RQ + NL * d][lc], &s_acc[RQ + NL * d + NL - 1][lc], m * kv[d], bad);
      }
      if constexpr (EMB) AC::add(&s_acc[RM][lc], &s_acc[RM + NL - 1][lc], m, bad);
    };
#pragma unroll
    for (int q = 0; q < TQ; ++q)
      if (tid + (uint32_t)(q * TT) < nreg) {
        double kv[3] = {0.0, 0.0, 0.0};
        if constexpr (AT) {
#pragma unroll
          for (int d = 0; d < 3; ++d) kv[d] = s_dv[d][tid + (uint32_t)(q * TT)];
        }
        sum_mom(lcs[q], v[q], mass_of(tg[q]), kv);
      }
    for (uint32_t k = TREG + tid; k < cnt; k += TT) {
      VT vv[3];
      uint32_t tag;
      load_vt<FORM>(In, k, vv, tag);
      const double m = mass_of(tag);
      double kv[3] = {0.0, 0.0, 0.0};
      if constexpr (AT) at_kick_tail<FORM>(tag - B.tag0, A.step, B.k0, B.k1, sqrt(B.kT / m), kv);
      sum_mom(lc_at(k), vv, m, kv);
    }
    __syncthreads();

    // ---- per cell: u (cell threads)
    auto cell_mass = [&](uint32_t l, uint32_t nc) -> double {
      if constexpr (EMB) return AC::value(s_acc[RM][l], s_acc[RM + NL - 1][l]);
      else return (double)nc * B.mass;
    };
    const uint32_t nc = cthr && cok ? s_cnt[tid] : 0u;
    // the cell's Gamma draw, now that N_c is known (on its own waves beside
    // the centre-of-mass velocities when the tile allows)
    if constexpr (THERMO) {
      if (gthr) {
        const uint32_t ng = s_cnt[gl];  // 0 for a cell outside the box
        uint32_t pend = 0u;
        double eh = -1.0;
        if (ng >= 2u) {
          double g[GPRE], lu[GPRE];
#pragma unroll
          for (int j = 0; j < GPRE; ++j) {
            g[j] = s_gam[2 * j][gl];
            lu[j] = s_gam[2 * j + 1][gl];
          }
          eh = gamma_first2(ng, g, lu, B.kT);
          if (eh < 0.0) {
            pend = 1u;
            s_anyp = 1u;
          }
        }
        s_ehat[gl] = eh;
        s_pend[gl] = pend;
      }
    }
    if (cthr) {
      double u[3] = {0.0, 0.0, 0.0};
      if (nc > 0u) {
        const double M = cell_mass(tid, nc);
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] = AC::value(s_acc[RP + NL * d][tid], s_acc[RP + NL * d + NL - 1][tid]) / M;
      }
      s_u[0][tid] = u[0];
      s_u[1][tid] = u[1];
      s_u[2][tid] = u[2];
      if constexpr (AT) {
        // mass-weighted mean random velocity of the cell, in s_ax
        const double M = nc > 0u ? cell_mass(tid, nc) : 1.0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
          s_ax[d][tid] = nc > 0u ? AC::value(s_acc[RQ + NL * d][tid], s_acc[RQ + NL * d + NL - 1][tid]) / M : 0.0;
      }
    }

    double ek = 0.0;
    if constexpr (EK) {
      __syncthreads();
      auto sum_energy = [&](uint32_t lc, const VT vv[3], double m) {
        const double dx = (double)vv[0] - s_u[0][lc], dy = (double)vv[1] - s_u[1][lc],
                     dz = (double)vv[2] - s_u[2][lc];
        AC::add(&s_acc[RE][lc], &s_acc[RE + NL - 1][lc], m * (dx * dx + dy * dy + dz * dz), bad);
      };
#pragma unroll
      for (int q = 0; q < TQ; ++q)
        if (tid + (uint32_t)(q * TT) < nreg) sum_energy(lcs[q], v[q], mass_of(tg[q]));
      for (uint32_t k = TREG + tid; k < cnt; k += TT) {
        VT vv[3];
        load_vel<FORM>(In, k, vv);
        sum_energy(lc_at(k), vv, mass_of(load_tag<FORM>(In, k)));
      }
      __syncthreads();
      if (cthr) ek = 0.5 * AC::value(s_acc[RE][tid], s_acc[RE + NL - 1][tid]);
    }

    // ---- per cell: xi (cell threads)
    if (cthr) {
      double xi = 1.0;
      if constexpr (THERMO) {
        // a pending draw is finished here when no particle follows (MODE_DIAG),
        // else after the main pass
        double ehat = s_ehat[tid];
        if constexpr (MODE == MODE_DIAG)
          if (s_pend[tid]) ehat = gamma_finish(nc, gcell, A.step, B, err);
        if (nc >= 2u && ek > 0.0) xi = sqrt(ehat / ek);
      }
      if constexpr (MODE == MODE_DIAG) {
        const double n[3] = {nc > 0u ? s_ax[0][tid] : 0.0, nc > 0u ? s_ax[1][tid] : 0.0,
                             nc > 0u ? s_ax[2][tid] : 0.0};
        if (cok) {
          const size_t oc = (size_t)B.cell0 + gcell;
          A.d_mass[oc] = nc > 0u ? cell_mass(tid, nc) : 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            A.d_mom[3u * oc + d] = AC::value(s_acc[RP + NL * d][tid], s_acc[RP + NL * d + NL - 1][tid]);
            A.d_axis[3u * oc + d] = n[d];
          }
          A.d_ek[oc] = ek;
          A.d_xi[oc] = xi;
        }
      } else if constexpr (THERMO) {
        s_xi[tid] = xi;
      }
    }

    if constexpr (MODE != MODE_DIAG) {
      __syncthreads();
      // particles of pending cells wait for the pass after the main one
      const bool anyp = THERMO && s_anyp != 0u;
      if constexpr (THERMO) {
        if (anyp) {
#pragma unroll
          for (int q = 0; q < TQ; ++q)
            if (tid + (uint32_t)(q * TT) < nreg && s_pend[lcs[q]]) lcs[q] |= LC_PEND;
        }
      }
      // ---- rotate (Alg. 1): v <- u + xi R(alpha, n) (v - u) in FP64, the
      // rotation by Rodrigues' formula from the axis, rounded once to the
      // storage precision
      auto rotate = [&](uint32_t lc, const VT vv[3], VT w[3], const double* kv) {
        if constexpr (AT) {
          // AT rule (eq. 4): u + dv - mean dv, rounded once
#pragma unroll
          for (int d = 0; d < 3; ++d) w[d] = (VT)((s_u[d][lc] + kv[d]) - s_ax[d][lc]);
          return;
        }
        const double u[3] = {s_u[0][lc], s_u[1][lc], s_u[2][lc]};
        const double n[3] = {s_ax[0][lc], s_ax[1][lc], s_ax[2][lc]};
        const double d[3] = {(double)vv[0] - u[0], (double)vv[1] - u[1], (double)vv[2] - u[2]};
        double r[3];
        rodrigues(n, B.ca, B.sa, B.omc, d, r);
        if constexpr (THERMO) {
          const double xi = s_xi[lc];
#pragma unroll
          for (int k = 0; k < 3; ++k) r[k] *= xi;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) w[k] = (VT)(u[k] + r[k]);
      };
      // LPOS scatter: per particle the local cell in the destination (bits
      // 0-7), bin (8-12) and rank within the bin (13-31), taken in the rotate
      // loop while the streamed position is in registers
      uint32_t info[LPOS ? TQ : 1];
      // a particle rotated outside the register-resident pass: stored in place
      // (MODE_COLLIDE), or streamed, binned and placed with one atomic
      auto finish_one = [&](uint32_t k, uint32_t lc, Pos<FORM>& rr, VT ww[3], uint32_t tag) {
        if constexpr (MODE == MODE_COLLIDE) {
          const Particles Out = tile_view<FORM>(A.out, tbase);
          store_part<FORM>(Out, k, rr, ww, tag);
          if (A.eslot_out) note_slot(A.eslot_out, B, tag, tbase + k);
        } else {
          if (streamed_in<MAY_EMB>(B, tag)) rr.stream(B, ww, err);
          scatter_one(rr, sh1.s, sh1.s32, ww, tag);
        }
      };
#pragma unroll
      for (int q = 0; q < TQ; ++q) {
        const uint32_t k = tid + (uint32_t)(q * TT);
        if constexpr (LPOS) info[q] = 0u;
        if (k < nreg && !(lcs[q] & LC_PEND)) {
          VT w[3];
          double kv[3] = {0.0, 0.0, 0.0};
          if constexpr (AT) {
#pragma unroll
            for (int d = 0; d < 3; ++d) kv[d] = s_dv[d][k];
          }
          rotate(lcs[q], v[q], w, kv);
          v[q][0] = w[0];
          v[q][1] = w[1];
          v[q][2] = w[2];
          if constexpr (LPOS) {
            Pos<FORM> rr;
            pos_from_lds(s_pos[k], FORM == 0 ? zq[q] : 0.0, rr);
            if constexpr (MODE == MODE_COLLIDE) {
              const Particles Out = tile_view<FORM>(A.out, tbase);
              store_part<FORM>(Out, k, rr, v[q], tg[q]);
              if (A.eslot_out) note_slot(A.eslot_out, B, tg[q], tbase + k);
            } else {
              if (streamed_in<MAY_EMB>(B, tg[q])) rr.stream(B, v[q], err);
              int c[3];
              rr.cell3(B, sh1.s, sh1.s32, c);
              uint32_t lcell;
              const uint32_t b = dest_bin(B, t3, c, lcell);
              const uint32_t rank = b < 27u ? atomicAdd(&s_bincnt[b], 1u) : 0u;
              info[q] = lcell | (b << 8) | (rank << 13);
              s_pos[k] = pos_to_lds(rr);
              if constexpr (FORM == 0) zq[q] = rr.x[2];
            }
          } else if constexpr (MODE == MODE_COLLIDE) {
            const Particles Out = tile_view<FORM>(A.out, tbase);
            store_part<FORM>(Out, k, r[q], v[q], tg[q]);
            if (A.eslot_out) note_slot(A.eslot_out, B, tg[q], tbase + k);
          } else {
            if (streamed_in<MAY_EMB>(B, tg[q])) r[q].stream(B, v[q], err);
          }
        }
      }
      if constexpr (MODE == MODE_COLLIDE_SCATTER) {
        if constexpr (LPOS) {
          // reserve the destination slots (one global atomic per bin), then
          // write each particle with its streamed position from LDS
          __syncthreads();
          if (tid < 27u && s_bincnt[tid] > 0u) s_base[tid] = atomicAdd(&A.cnt_out[s_btile[tid]], s_bincnt[tid]);
          __syncthreads();
#pragma unroll
          for (int q = 0; q < TQ; ++q) {
            const uint32_t k = tid + (uint32_t)(q * TT);
            if (k < nreg && !(lcs[q] & LC_PEND)) {
              Pos<FORM> rr;
              pos_from_lds(s_pos[k], FORM == 0 ? zq[q] : 0.0, rr);
              const uint32_t b = (info[q] >> 8) & 31u;
              uint32_t dt, slot;
              if (b < 27u) {
                dt = s_btile[b];
                slot = s_base[b] + (info[q] >> 13);
              } else {
                int c[3];
                rr.cell3(B, sh1.s, sh1.s32, c);
                dt = B.tile0 + tile_index(B, c);
                slot = atomicAdd(&A.cnt_out[dt], 1u);
              }
              if (slot < cap) put((size_t)dt * cap + slot, v[q], tg[q], rr, info[q] & 255u);
              else overflow();
            }
          }
        } else {
          scatter(sh1.s, sh1.s32, v);
        }
      }
      for (uint32_t k = TREG + tid; k < cnt; k += TT) {
        VT vv[3], ww[3];
        uint32_t tag;
        Pos<FORM> rr;
        const uint32_t lc = lc_at(k);
        if (THERMO && anyp && s_pend[lc]) continue;
        load_part<FORM>(In, k, rr, vv, tag);
        double kv[3] = {0.0, 0.0, 0.0};
        if constexpr (AT) at_kick_tail<FORM>(tag - B.tag0, A.step, B.k0, B.k1, sqrt(B.kT / mass_of(tag)), kv);
        rotate(lc, vv, ww, kv);
        finish_one(k, lc, rr, ww, tag);
      }

      // ---- pending cells: the cell threads finish their draws (the tile's
      // registers are free now), then the particles of those cells are read
      // again, rotated and placed one by one
      if constexpr (THERMO) {
        if (anyp) {
          if (cthr && s_pend[tid]) {
            bool ok;
            const uint32_t gc = cell_of(tid, ok);
            const double e = gamma_finish(s_cnt[tid], gc, A.step, B, err);
            const double ekc = 0.5 * AC::value(s_acc[RE][tid], s_acc[RE + NL - 1][tid]);
            s_xi[tid] = ekc > 0.0 ? sqrt(e / ekc) : 1.0;
          }
          __syncthreads();
          for (uint32_t k = tid; k < cnt; k += TT) {
            const uint32_t lc = lc_at(k);
            if (!s_pend[lc]) continue;
            VT vv[3], ww[3];
            uint32_t tag;
            Pos<FORM> rr;
            load_part<FORM>(In, k, rr, vv, tag);
            const double kv[3] = {0.0, 0.0, 0.0};
            rotate(lc, vv, ww, kv);
            finish_one(k, lc, rr, ww, tag);
          }
        }
      }
    }
  }
  if (bad) err |= ERR_FIXED_RANGE;
  if (err) atomicOr(&A.status[0], err);
}

// ------------------------------------------------- elementwise over slabs
// Valid slot k of tile T: k < cnt[T]. Grid: ntiles * ceil(cap / 256) blocks.
struct SlabIter {
  uint32_t T, k;
  size_t i;
  bool valid;
};
__device__ inline SlabIter slab_slot(const Slabs& S, const uint32_t* cnt) {
  const uint32_t per = (S.cap + 255u) / 256u;
  SlabIter s;
  s.T = blockIdx.x / per;
  s.k = (blockIdx.x % per) * 256u + threadIdx.x;
  s.i = (size_t)s.T * S.cap + s.k;
  s.valid = s.T < S.ntiles && s.k < min(cnt[s.T], S.cap);
  return s;
}

template <int FORM>
__global__ __launch_bounds__(256) void k_stream(Particles P, Slabs S, const uint32_t* cnt,
                                                uint32_t* status) {
  const SlabIter s = slab_slot(S, cnt);
  if (!s.valid) return;
  const Box& B = S.boxes[S.tile_box[s.T]];
  typename VelT<FORM>::T v[3];
  uint32_t tag;
  Pos<FORM> r;
  load_part<FORM>(P, s.i, r, v, tag);
  uint32_t e = 0;
  if (streamed(B, tag)) r.stream(B, v, e);
  store_part<FORM>(P, s.i, r, v, tag);
  if (e) atomicOr(&status[0], e);
}

// Cell of every particle (box-local index) for the per-box shifts sh, in tag
// order, and the occupancy (at cell0 + cell).
template <int FORM>
__global__ __launch_bounds__(256) void k_cells(Particles P, Slabs S, const uint32_t* cnt,
                                               const ShiftEntry* __restrict__ sh,
                                               int32_t* cell_of_tag, uint32_t* counts) {
  const SlabIter s = slab_slot(S, cnt);
  if (!s.valid) return;
  const uint32_t bx = S.tile_box[s.T];
  const Box& B = S.boxes[bx];
  Pos<FORM> r;
  r.load(P, s.i);
  int c[3];
  r.cell3(B, sh[bx].s, sh[bx].s32, c);
  const uint32_t cell = cell_index(B, c);
  if (cell_of_tag) cell_of_tag[load_tag<FORM>(P, s.i)] = (int32_t)cell;
  if (counts) atomicAdd(&counts[B.cell0 + cell], 1u);
}

// Mass and momentum of every cell of the unshifted grid (the particle's home
// cell), for the cell-averaged velocity field: exact fixed-point sums in
// global memory, 8 words per cell (P_x, P_y, P_z, M, two limbs each), at
// acc[8 (cell0 + cell) ...]. Integer atomics commute, so the sums do not
// depend on the order in which particles are visited.
template <int FORM, bool EMB>
__global__ __launch_bounds__(256) void k_field(Particles P, Slabs S, const uint32_t* cnt,
                                               const double* __restrict__ emb_mass,
                                               unsigned long long* acc, uint32_t* status) {
  const SlabIter s = slab_slot(S, cnt);
  if (!s.valid) return;
  const Box B = S.boxes[S.tile_box[s.T]];
  Pos<FORM> r;
  r.load(P, s.i);
  int c[3];
  r.home3(B, c);
  const uint32_t cell = B.cell0 + cell_index(B, c);
  typename VelT<FORM>::T v[3];
  load_vel<FORM>(P, s.i, v);
  double m = B.mass;
  if constexpr (EMB) {
    const uint32_t i = load_tag<FORM>(P, s.i) - B.tag0;
    if (i >= B.n_solvent) m = emb_mass[i - B.n_solvent];
  }
  bool bad = false;
  const double x[4] = {m * (double)v[0], m * (double)v[1], m * (double)v[2], m};
  unsigned long long* a = acc + 8ull * cell;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    long long hi, lo;
    fx_split(x[q], hi, lo, bad);
    atomicAdd(&a[2 * q], (unsigned long long)hi);
    atomicAdd(&a[2 * q + 1], (unsigned long long)lo);
  }
  if (bad) atomicOr(&status[0], ERR_FIXED_RANGE);
}

// u = P / M per cell (0 where the cell is empty), and M.
__global__ void k_field_finish(const unsigned long long* __restrict__ acc, uint64_t ncells,
                               double* __restrict__ u, double* __restrict__ mass) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i >= ncells) return;
  const unsigned long long* a = acc + 8ull * i;
  double w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Fx f;
    f.hi = (long long)a[2 * q];
    f.lo = (long long)a[2 * q + 1];
    w[q] = fx_value(f);
  }
  if (u)
    for (int d = 0; d < 3; ++d) u[3 * i + d] = w[3] > 0.0 ? w[d] / w[3] : 0.0;
  if (mass) mass[i] = w[3];
}

// Grid shifts of steps n0 .. n0 + nsteps - 1 for every box: entry
// [k * nbox + b] (zero when the shift is off).
__global__ void k_shifts(const Box* __restrict__ boxes, uint32_t nbox, uint32_t n0,
                         uint32_t nsteps, int32_t on, ShiftEntry* __restrict__ out) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= nbox * nsteps) return;
  const uint32_t b = i % nbox, k = i / nbox;
  const Box& B = boxes[b];
  ShiftEntry e;
  if (on) {
    grid_shift(B.k0, B.k1, n0 + k, B.a, e.s);
  } else {
    e.s[0] = e.s[1] = e.s[2] = 0.0;
  }
  for (int d = 0; d < 3; ++d) e.s32[d] = (float)e.s[d];
  e.pad = 0.0f;
  out[i] = e;
}

// Net momentum, kinetic energy and mass in fixed point: block sums in LDS
// (integer, so exact), then 64-bit atomics, which commute.
template <int FORM, bool EMB>
__global__ __launch_bounds__(256) void k_totals(Particles P, Slabs S, const uint32_t* cnt,
                                                const double* __restrict__ emb_mass,
                                                long long* tot, uint32_t* status) {
  __shared__ long long red[10][256];
  Fx acc[5] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}, {0, 0}};
  bool bad = false;
  const SlabIter s = slab_slot(S, cnt);
  // a block covers part of one tile, so of one box; totals per box
  const uint32_t bx = S.tile_box[min(s.T, S.ntiles - 1u)];
  const Box& B = S.boxes[bx];
  if (s.valid) {
    typename VelT<FORM>::T vs[3];
    load_vel<FORM>(P, s.i, vs);
    const double v[3] = {(double)vs[0], (double)vs[1], (double)vs[2]};
    double m = B.mass;
    if constexpr (EMB) {
      const uint32_t i = load_tag<FORM>(P, s.i) - B.tag0;
      if (i >= B.n_solvent) m = emb_mass[i - B.n_solvent];
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
    atomicAdd(reinterpret_cast<unsigned long long*>(&tot[10u * bx + threadIdx.x]),
              (unsigned long long)red[threadIdx.x][0]);
  if (bad) atomicOr(&status[0], ERR_FIXED_RANGE);
}

// ------------------------------------------------------------ state I/O
// Row-major N x 3 doubles (tag order) -> internal form, placed in the slab of
// the tile of the particle's home cell. Pass 1 (PLACE == false) only counts
// per tile and checks the box; pass 2 writes.
// A position in [0, L) in the storage form: FP64 as is; FP32 as home cell
// floor(x / a) (clamped) and the FP32 offset x - h a, an offset that rounds
// up to a moving to the next cell at offset 0.
template <int FORM>
__device__ inline void to_form(const Box& B, const double x[3], Pos<FORM>& r) {
  if constexpr (FORM == 0) {
    r.x[0] = x[0];
    r.x[1] = x[1];
    r.x[2] = x[2];
  } else {
    int hh[3];
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
      hh[d] = hd;
      r.o[d] = o;
    }
    r.hp = pack_home(hh[0], hh[1], hh[2]);
  }
}

template <int FORM, bool PLACE>
__global__ __launch_bounds__(256) void k_import(Particles P, Box B, uint32_t cap,
                                                const double* __restrict__ pos,
                                                const double* __restrict__ vel,
                                                uint32_t n, uint32_t tag0, uint32_t* cnt,
                                                uint32_t* bad_pos, uint32_t* eslot) {
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
  using VT = typename VelT<FORM>::T;
  const VT w[3] = {(VT)v[0], (VT)v[1], (VT)v[2]};
  to_form<FORM>(B, x, r);
  int c[3];
  r.home3(B, c);
  const uint32_t T = B.tile0 + tile_index(B, c);
  const uint32_t slot = atomicAdd(&cnt[T], 1u);
  if constexpr (PLACE) {
    if (slot < cap) {
      const size_t j = (size_t)T * cap + slot;
      store_part<FORM>(P, j, r, w, tag0 + t);
      if (eslot) note_slot(eslot, B, tag0 + t, j);
    } else {
      atomicOr(bad_pos, 2u);
    }
  }
}

// Internal form -> row-major N x 3 doubles in tag order.
template <int FORM>
// pos (if non-null) and vel (if non-null) of every particle, in tag order
__global__ __launch_bounds__(256) void k_export(Particles P, Slabs S, const uint32_t* cnt,
                                                double* __restrict__ pos,
                                                double* __restrict__ vel) {
  const SlabIter s = slab_slot(S, cnt);
  if (!s.valid) return;
  const Box& B = S.boxes[S.tile_box[s.T]];
  typename VelT<FORM>::T v[3];
  uint32_t t;
  Pos<FORM> r;
  load_part<FORM>(P, s.i, r, v, t);
  if (pos) {
    if constexpr (FORM == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) pos[3ull * t + d] = r.x[d];
    } else {
      int h[3];
      unpack_home(r.hp, h[0], h[1], h[2]);
#pragma unroll
      for (int d = 0; d < 3; ++d) pos[3ull * t + d] = (double)h[d] * B.a + (double)r.o[d];
    }
  }
  if (vel) {
#pragma unroll
    for (int d = 0; d < 3; ++d) vel[3ull * t + d] = (double)v[d];
  }
}

// Velocities handed from one buffer to the other through a tag-indexed
// array tmp (3 per tag, storage precision): k_vel_by_tag fills tmp from the
// slots of one buffer, k_vel_from_tag writes them into the slots that hold
// the same tags in the other.
template <int FORM>
__global__ __launch_bounds__(256) void k_vel_by_tag(Particles P, Slabs S, const uint32_t* cnt,
                                                    typename VelT<FORM>::T* __restrict__ tmp) {
  const SlabIter s = slab_slot(S, cnt);
  if (!s.valid) return;
  typename VelT<FORM>::T v[3];
  uint32_t t;
  load_vt<FORM>(P, s.i, v, t);
#pragma unroll
  for (int d = 0; d < 3; ++d) tmp[3ull * t + d] = v[d];
}

template <int FORM>
__global__ __launch_bounds__(256) void k_vel_from_tag(Particles P, Slabs S, const uint32_t* cnt,
                                                      const typename VelT<FORM>::T* __restrict__ tmp) {
  const SlabIter s = slab_slot(S, cnt);
  if (!s.valid) return;
  typename VelT<FORM>::T v[3];
  uint32_t t;
  Pos<FORM> r;
  load_part<FORM>(P, s.i, r, v, t);
#pragma unroll
  for (int d = 0; d < 3; ++d) v[d] = tmp[3ull * t + d];
  store_vel<FORM>(P, s.i, r, v, t);
}

// Copy the valid slots of every tile from slabs of capacity old_cap to slabs
// of capacity S.cap (S.cap >= old_cap); used when slabs are enlarged.
template <int FORM>
__global__ __launch_bounds__(256) void k_repack(Particles src, Particles dst, Slabs S,
                                                uint32_t old_cap, const uint32_t* cnt, uint32_t* eslot) {
  const uint32_t per = (old_cap + 255u) / 256u;
  const uint32_t T = blockIdx.x / per;
  const uint32_t k = (blockIdx.x % per) * 256u + threadIdx.x;
  if (T >= S.ntiles || k >= min(cnt[T], old_cap)) return;
  const size_t i = (size_t)T * old_cap + k, j = (size_t)T * S.cap + k;
  typename VelT<FORM>::T v[3];
  uint32_t tag;
  Pos<FORM> r;
  load_part<FORM>(src, i, r, v, tag);
  store_part<FORM>(dst, j, r, v, tag);
  if (eslot) note_slot(eslot, S.boxes[S.tile_box[T]], tag, j);
}

// --------------------------------------------------------- test kernels
__global__ void k_philox(const U4* __restrict__ ctr, uint32_t n, uint32_t k0,
                         uint32_t k1, U4* __restrict__ out) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) out[i] = philox4x32_10(ctr[i], k0, k1);
}

// Streaming copy, 16-byte vectors, nontemporal, grid-stride.
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * 256u + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * 256u)
    nt_store(dst + i, nt_load(src + i));
}

// The same copy with four vectors per thread and iteration, all four loaded
// before any is stored (more loads in flight per wave).
__global__ __launch_bounds__(256) void k_copy16x4(const uint4* __restrict__ src,
                                                  uint4* __restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * 256u;
  size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = nt_load(src + i), b = nt_load(src + i + stride);
    const uint4 c = nt_load(src + i + 2 * stride), d = nt_load(src + i + 3 * stride);
    nt_store(dst + i, a);
    nt_store(dst + i + stride, b);
    nt_store(dst + i + 2 * stride, c);
    nt_store(dst + i + 3 * stride, d);
  }
  for (; i < n16; i += stride) nt_store(dst + i, nt_load(src + i));
}

__global__ void k_copy1(const unsigned char* __restrict__ src,
                        unsigned char* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace mpcd
