// Exchange of embedded particles (solutes) between the slabs and row-major
// arrays: export, import, and the handover into a prepared binning. Kept
// apart from the step kernel.
#pragma once

#include "mpcd_kernels.hpp"

namespace mpcd {

// The position-bearing words of record j only: the FP32 form's position
// word; the FP64 form's {x, y} and {z, v_x} words (v_x rewritten with w[0]).
template <int FORM, class I>
__device__ inline void store_pos(const Particles& P, I j, const Pos<FORM>& r,
                                 const typename VelT<FORM>::T w[3]) {
  if constexpr (FORM == 0) {
    st(P.wa, j, make_double2(r.x[0], r.x[1]));
    st(P.wb, j, make_double2(r.x[2], w[0]));
  } else {
    st(P.ra, j, make_uint4(r.hp, __float_as_uint(r.o[0]), __float_as_uint(r.o[1]), __float_as_uint(r.o[2])));
  }
}

// Embedded particles out of / into the slabs, rows tag - n_solvent of
// row-major n_emb x 3 doubles: the exchange with an external MD integrator
// between collisions. One thread per embedded particle of box B (the only
// box that has them), found through the slot index of a buffer (nslots
// slots); export writes pos and vel where they are non-null, import updates
// the slot in place, and the next binning moves the particle to the tile of
// its new position. A slot out of range or not holding the expected tag sets
// bit 2 of *flag and is left alone.
template <int FORM>
__global__ __launch_bounds__(256) void k_emb_export(Particles P, Box B, const uint32_t* __restrict__ eslot,
                                                    uint32_t n, size_t nslots, double* __restrict__ pos,
                                                    double* __restrict__ vel, uint32_t* flag) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const size_t j = eslot[i];
  if (j >= nslots) {
    atomicOr(flag, 4u);
    return;
  }
  typename VelT<FORM>::T v[3];
  uint32_t t;
  Pos<FORM> r;
  load_part<FORM>(P, j, r, v, t);
  if (t != B.tag0 + B.n_solvent + i) {
    atomicOr(flag, 4u);
    return;
  }
  const size_t row = 3ull * i;
  if (pos) {
    if constexpr (FORM == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) pos[row + d] = r.x[d];
    } else {
      int h[3];
      unpack_home(r.hp, h[0], h[1], h[2]);
#pragma unroll
      for (int d = 0; d < 3; ++d) pos[row + d] = (double)h[d] * B.a + (double)r.o[d];
    }
  }
  if (vel) {
#pragma unroll
    for (int d = 0; d < 3; ++d) vel[row + d] = (double)v[d];
  }
}

// The split state in one pass: positions from the current buffer Pc,
// velocities from the prepared buffer Pp, each through its own slot index.
template <int FORM>
__global__ __launch_bounds__(256) void k_emb_export_split(Particles Pc, Particles Pp, Box B,
                                                          const uint32_t* __restrict__ eslot_c,
                                                          const uint32_t* __restrict__ eslot_p, uint32_t n,
                                                          size_t nslots, double* __restrict__ pos,
                                                          double* __restrict__ vel, uint32_t* flag) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const size_t jc = eslot_c[i], jp = eslot_p[i];
  const uint32_t t = B.tag0 + B.n_solvent + i;
  if (jc >= nslots || jp >= nslots || load_tag<FORM>(Pc, jc) != t) {
    atomicOr(flag, 4u);
    return;
  }
  typename VelT<FORM>::T v[3];
  uint32_t tp;
  load_vt<FORM>(Pp, jp, v, tp);
  if (tp != t) {
    atomicOr(flag, 4u);
    return;
  }
  const size_t row = 3ull * i;
  if constexpr (FORM == 0) {
    const double2 a = ld(Pc.wa, jc), b = ld(Pc.wb, jc);
    pos[row] = a.x;
    pos[row + 1] = a.y;
    pos[row + 2] = b.x;
  } else {
    const uint4 a = ld(Pc.ra, jc);
    int h[3];
    unpack_home(a.x, h[0], h[1], h[2]);
    const float o[3] = {__uint_as_float(a.y), __uint_as_float(a.z), __uint_as_float(a.w)};
#pragma unroll
    for (int d = 0; d < 3; ++d) pos[row + d] = (double)h[d] * B.a + (double)o[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) vel[row + d] = (double)v[d];
}

// Positions outside [0, L) set bit 0 of *flag and are not stored.
template <int FORM>
__global__ __launch_bounds__(256) void k_emb_import(Particles P, Box B, const uint32_t* __restrict__ eslot,
                                                    uint32_t n, size_t nslots, const double* __restrict__ pos,
                                                    const double* __restrict__ vel, uint32_t* flag) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const size_t j = eslot[i];
  const uint32_t t = B.tag0 + B.n_solvent + i;
  if (j >= nslots || load_tag<FORM>(P, j) != t) {
    atomicOr(flag, 4u);
    return;
  }
  const size_t row = 3ull * i;
  double x[3];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d] = pos[row + d];
    bad |= !(x[d] >= 0.0 && x[d] < B.L[d]);
  }
  if (bad) {
    atomicOr(flag, 1u);
    return;
  }
  using VT = typename VelT<FORM>::T;
  const VT w[3] = {(VT)vel[row], (VT)vel[row + 1], (VT)vel[row + 2]};
  Pos<FORM> r;
  to_form<FORM>(B, x, r);
  store_part<FORM>(P, j, r, w, t);
}

// Handover of embedded particles into a prepared binning (the buffer the
// last collision scattered into, binned for the next step with that step's
// shift): O(embedded particles), the solvent's binning is kept.
//   k_emb_rebin   per particle: the new position into its slot of the
//                 current buffer (whose velocities are not read while the
//                 binning is prepared); its cell under the prepared step's
//                 shift; if that
//                 cell lies in the tile whose slab holds the particle, the
//                 prepared slot is updated in place, else the particle is a
//                 mover (listed, and linked into its old tile's departures);
//   k_emb_depart  per tile with departures (run by the thread of its list
//                 head): the departing slots are marked, then filled with the
//                 tile's last non-departing particles, and the count shrinks;
//   k_emb_arrive  per mover: a slot at the end of its new tile's slab.
// A slot or tag that does not match the slot index sets bit 2 of *flag, a
// position outside [0, L) bit 0 (the particle keeps its old state); a full
// destination slab sets bit 3 and leaves the mover out of the prepared buffer
// (the caller then gives the prepared binning up).
constexpr uint32_t kNoTag = 0xFFFFFFFFu;

template <int FORM>
__device__ inline void set_tag(const Particles& P, size_t j, uint32_t t) {
  if constexpr (FORM == 0) P.tag[j] = t;
  else reinterpret_cast<uint32_t*>(P.rb)[4 * j + 3] = t;
}

template <int FORM>
__device__ inline bool emb_input(const Box& B, uint32_t i, const double* __restrict__ pos,
                                 const double* __restrict__ vel, Pos<FORM>& r,
                                 typename VelT<FORM>::T w[3]) {
  double x[3];
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    x[d] = pos[3ull * i + d];
    bad |= !(x[d] >= 0.0 && x[d] < B.L[d]);
  }
  if (bad) return false;
  using VT = typename VelT<FORM>::T;
#pragma unroll
  for (int d = 0; d < 3; ++d) w[d] = (VT)vel[3ull * i + d];
  to_form<FORM>(B, x, r);
  return true;
}

template <int FORM>
__device__ inline uint32_t emb_tile(const Box& B, const ShiftEntry& sh, const Pos<FORM>& r,
                                    uint32_t& lcell) {
  int c[3];
  r.cell3(B, sh.s, sh.s32, c);
  lcell = local_cell(B, c);
  return B.tile0 + tile_index(B, c);
}

template <int FORM>
__global__ __launch_bounds__(256) void k_emb_rebin(Particles Pp, Particles Pc, Box B, const ShiftEntry* sh,
                                                   const uint32_t* __restrict__ eslot_p,
                                                   const uint32_t* __restrict__ eslot_c, uint32_t n,
                                                   size_t nslots, uint32_t cap,
                                                   const double* __restrict__ pos,
                                                   const double* __restrict__ vel, int32_t* dep_head,
                                                   int32_t* dep_next, uint32_t* movers,
                                                   uint32_t* nmovers, uint32_t* flag) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = B.tag0 + B.n_solvent + i;
  const size_t jp = eslot_p[i], jc = eslot_c[i];
  if (jp >= nslots || jc >= nslots || load_tag<FORM>(Pp, jp) != t || load_tag<FORM>(Pc, jc) != t) {
    atomicOr(flag, 4u);
    return;
  }
  Pos<FORM> r;
  typename VelT<FORM>::T w[3];
  if (!emb_input<FORM>(B, i, pos, vel, r, w)) {
    atomicOr(flag, 1u);
    return;
  }
  store_pos<FORM>(Pc, jc, r, w);
  uint32_t lcell;
  const uint32_t T = emb_tile<FORM>(B, sh[0], r, lcell);
  const uint32_t T0 = (uint32_t)(jp / cap);
  if (T == T0) {
    store_part<FORM>(Pp, jp, r, w, t);
  } else {
    movers[atomicAdd(nmovers, 1u)] = i;
    dep_next[i] = atomicExch(&dep_head[T0], (int32_t)i);
  }
}

template <int FORM>
__global__ __launch_bounds__(256) void k_emb_depart(Particles Pp, Box B, uint32_t* eslot_p, uint32_t cap,
                                                    uint32_t* cnt_p, const uint32_t* __restrict__ movers,
                                                    const uint32_t* __restrict__ nmovers, int32_t* dep_head,
                                                    const int32_t* __restrict__ dep_next) {
  const uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= *nmovers) return;
  const uint32_t i = movers[k];
  const uint32_t T = eslot_p[i] / cap;
  if (dep_head[T] != (int32_t)i) return;  // the list head's thread takes the tile
  const size_t base = (size_t)T * cap;
  uint32_t m = 0;
  for (int32_t b = (int32_t)i; b >= 0; b = dep_next[b]) {
    set_tag<FORM>(Pp, eslot_p[b], kNoTag);
    ++m;
  }
  const uint32_t n = cnt_p[T], keep = n - m;
  uint32_t top = n;  // slots [top, n) are done
  for (int32_t b = (int32_t)i; b >= 0; b = dep_next[b]) {
    const size_t j = eslot_p[b];
    if (j - base >= keep) continue;  // above the kept range: dropped with the count
    size_t s;
    do {
      --top;
      s = base + top;
    } while (load_tag<FORM>(Pp, s) == kNoTag);
    typename VelT<FORM>::T v[3];
    uint32_t tag;
    Pos<FORM> r;
    load_part<FORM>(Pp, s, r, v, tag);
    store_part<FORM>(Pp, j, r, v, tag);
    note_slot(eslot_p, B, tag, j);
  }
  cnt_p[T] = keep;
  dep_head[T] = -1;
}

template <int FORM>
__global__ __launch_bounds__(256) void k_emb_arrive(Particles Pp, Box B, const ShiftEntry* sh,
                                                    uint32_t* eslot_p, uint32_t cap, uint32_t* cnt_p,
                                                    const uint32_t* __restrict__ movers,
                                                    const uint32_t* __restrict__ nmovers,
                                                    const double* __restrict__ pos,
                                                    const double* __restrict__ vel, uint32_t* flag) {
  const uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= *nmovers) return;
  const uint32_t i = movers[k];
  Pos<FORM> r;
  typename VelT<FORM>::T w[3];
  (void)emb_input<FORM>(B, i, pos, vel, r, w);  // checked by k_emb_rebin
  uint32_t lcell;
  const uint32_t T = emb_tile<FORM>(B, sh[0], r, lcell);
  const uint32_t slot = atomicAdd(&cnt_p[T], 1u);
  if (slot >= cap) {
    atomicSub(&cnt_p[T], 1u);
    atomicOr(flag, 8u);
    return;
  }
  const size_t j = (size_t)T * cap + slot;
  store_part<FORM>(Pp, j, r, w, B.tag0 + B.n_solvent + i);
  eslot_p[i] = (uint32_t)j;
}

}  // namespace mpcd
