// libmpcd: host side of the C ABI declared in include/mpcd.h.
//
// A context holds one box, or several independent boxes stepped together
// (a batch). It owns every device buffer (stream-ordered allocations on its
// stream, freed the same way) and enqueues all work on that one HIP stream.
// Particles live in fixed-capacity per-tile slabs (see mpcd_kernels.hpp); the
// tiles of all boxes share the slab arrays, and every launch covers all of
// them. A call to mpcd_step launches, unless the last call left the binning
// prepared, one stream+bin kernel and then one tile kernel per step (the
// thermostat's draws included); it waits for the stream at its end to confirm
// that no slab overflowed. If one did, the input of the failing launch is
// still intact: the slabs are enlarged, that input is repacked, and the
// launches are replayed from there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mpcd.h"
#include "mpcd_kernels.hpp"
#include "mpcd_emb.hpp"
#include "mpcd_md.hpp"

using namespace mpcd;

namespace {

thread_local std::string g_err;

// Allocation-failure injection for tests of the cleanup paths: after
// g_fail_after more successful device allocations, g_fail_count fail.
std::atomic<int64_t> g_fail_after{-1}, g_fail_count{0};

bool inject_alloc_failure() {
  if (g_fail_after.load() < 0) return false;
  if (g_fail_after.fetch_sub(1) > 0) return false;
  g_fail_after.store(0);
  if (g_fail_count.fetch_sub(1) > 0) return true;
  g_fail_after.store(-1);
  g_fail_count.store(0);
  return false;
}

mpcd_status fail(mpcd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(e_ == hipErrorOutOfMemory ? MPCD_ENOMEM : MPCD_EHIP,             \
                  "%s failed: %s", #expr, hipGetErrorString(e_));                  \
  } while (0)

#define ST_TRY(expr)                    \
  do {                                  \
    mpcd_status s_ = (expr);            \
    if (s_ != MPCD_OK) return s_;       \
  } while (0)

enum class Phase { Idle, Streamed, Binned };

// One queued kernel of a stepping call.
// CollideLast: the collide + scatter that ends a call. The input buffer stays
// current: it keeps the positions (and cells) of the state after the
// collision, while the output holds that state's velocities, streamed and
// binned for the next step (see `split`).
enum class Op { BinStream, Bin, CollideScatter, Collide, CollideLast };
struct Launch {
  Op op;
  uint64_t step;
};

constexpr uint32_t kGrid = 256;  // threads per block of the elementwise kernels
// slots per tile stay below 2^28: a slot's byte offset inside its tile's
// slab then fits 32 bits for every element size
constexpr uint32_t kMaxCap = 1u << 28;

inline uint32_t blocks_for(uint64_t n, uint32_t per) {
  return (uint32_t)((n + per - 1) / per);
}

inline uint32_t round_up(uint64_t x, uint32_t m) { return (uint32_t)(((x + m - 1) / m) * m); }

}  // namespace

struct mpcd_ctx_s {
  mpcd_params p{};                 // settings shared by all boxes (box 0's parameters)
  int form = 0;
  uint32_t nbox = 0;
  uint32_t n_emb = 0, N = 0;       // embedded particles (box 0 only), all particles
  std::vector<Box> boxes;          // host copies of the per-box constants
  std::vector<uint32_t> box_n;     // particles per box
  Slabs S{};                       // device view of the layout
  uint64_t ncells = 0;             // cells of all boxes
  int cpt = 64;  // cells per tile rounded up to 64/128/256 (kernel template)
  hipStream_t stream = nullptr;
  bool own_stream = false;

  std::vector<void*> allocs;       // everything but the slabs and the shift table
  std::vector<void*> slab_allocs;  // the two particle buffers
  Particles buf[2]{};
  int cur = 0;
  uint32_t* cnt[3] = {nullptr, nullptr, nullptr};
  int ci = 0;                      // cnt[ci] describes buf[cur]
  double* emb_mass = nullptr;
  uint32_t* flag = nullptr;        // one word a host call checks after a kernel (range errors)
  uint32_t* eslot[2] = {nullptr, nullptr};  // slot of each embedded particle in buf[0], buf[1]
  // handover of embedded particles into a prepared binning (allocated on
  // first use): departures per tile (list heads, -1 when empty), links,
  // movers and their count
  int32_t* dep_head = nullptr;
  int32_t* dep_next = nullptr;
  uint32_t* movers = nullptr;
  uint32_t* nmovers = nullptr;
  uint32_t* status = nullptr;      // [0] errors, [1] overflow, [2] failing launch
  long long* tot = nullptr;        // fixed-point totals, 10 words per box

  ShiftEntry* shifts = nullptr;    // grid shifts of steps shift_n0 .., [step][box]
  uint64_t shift_cap = 0, shift_n0 = 0, shift_count = 0;
  const ShiftEntry* shift_view = nullptr;  // the table the next launches read (shifts, or
                                           // the library's static one in mpcd_step_noalloc)
  int device = 0;                  // the device current at create

  uint64_t step = 0;
  uint64_t last_bin_step = 0;
  Phase phase = Phase::Idle;
  bool have_bin = false;
  // buf[1 - cur] with cnt[(ci + 1) % 3] holds the current state streamed and
  // binned for step `step` (left by the last mpcd_step), so the next
  // mpcd_step starts with its collision
  bool pre = false;
  // the current state is split over the buffers: positions and cells in
  // buf[cur], velocities (by tag) only in buf[1 - cur] (pre is then true);
  // readbacks join the two, and materialize() copies the velocities back
  // before anything needs buf[cur] whole
  bool split = false;
  int64_t regrows = 0;
  uint64_t handovers[2] = {0, 0};  // solute handovers into a prepared binning: kept, given up

  // graph launches: the tile launches of a stepping call are captured into
  // a graph and replayed; the executable graph is kept and updated in place
  // by the next call's capture when its shape allows
  bool graph = false;
  hipGraphExec_t gexec = nullptr;
  uint64_t graph_inst = 0, graph_upd = 0;

  int32_t prof_every = 0;          // time one launch in every prof_every of a kind (0: off)
  uint64_t prof_seen[2] = {0, 0};
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[2];

  // Device memory comes from the stream-ordered allocator on the context's
  // stream: allocating and freeing never waits for the whole device, so
  // contexts on other streams (concurrent requests) keep running.
  hipError_t alloc(void** q, size_t bytes) {
    if (inject_alloc_failure()) {
      *q = nullptr;
      return hipErrorOutOfMemory;
    }
    return hipMallocAsync(q, bytes ? bytes : 256, stream);
  }
  void release(void* q) {
    if (q) (void)hipFreeAsync(q, stream);
  }
  void* dalloc(size_t bytes) {
    void* q = nullptr;
    if (alloc(&q, bytes) != hipSuccess) return nullptr;
    allocs.push_back(q);
    return q;
  }
};

namespace {

mpcd_status check_ctx(mpcd_ctx c) {
  if (!c) return fail(MPCD_EINVAL, "null context");
  return MPCD_OK;
}

mpcd_status take_err(mpcd_ctx c) {
  uint32_t e = 0;
  HIP_TRY(hipMemcpyAsync(&e, c->status, sizeof e, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (e) {
    HIP_TRY(hipMemsetAsync(c->status, 0, sizeof e, c->stream));
    return fail(MPCD_ERANGE, "kernel range check failed (flags 0x%x: %s%s%s)", e,
                (e & ERR_STREAM_RANGE) ? "displacement >= box length; " : "",
                (e & ERR_FIXED_RANGE) ? "value outside fixed-point range; " : "",
                (e & ERR_GAMMA_CAP) ? "Gamma sampler attempt cap; " : "");
  }
  return MPCD_OK;
}

// Host copy of box b's shift for step n (the kernels read the device table).
void shift_for(const mpcd_ctx c, uint32_t b, uint64_t n, double s[3]) {
  if (c->p.grid_shift) {
    grid_shift(c->boxes[b].k0, c->boxes[b].k1, (uint32_t)n, c->boxes[b].a, s);
  } else {
    s[0] = s[1] = s[2] = 0.0;
  }
}

// Fill the device shift table with steps n0 .. n0 + count - 1 of every box.
mpcd_status ensure_shifts(mpcd_ctx c, uint64_t n0, uint64_t count) {
  // the context's own table already holds these steps (the shifts depend on
  // the seed, the step and the box only)
  if (c->shifts && c->shift_view == c->shifts && n0 >= c->shift_n0 &&
      n0 + count <= c->shift_n0 + c->shift_count)
    return MPCD_OK;
  const uint64_t need = count * c->nbox;
  if (need > c->shift_cap) {
    if (c->shifts) {
      c->release(c->shifts);  // stream-ordered: after the launches that read it
      c->shifts = nullptr;
      c->shift_cap = 0;
    }
    const uint64_t cap = std::max<uint64_t>(need, 64);
    HIP_TRY(c->alloc((void**)&c->shifts, cap * sizeof(ShiftEntry)));
    c->shift_cap = cap;
  }
  k_shifts<<<blocks_for(need, 256), 256, 0, c->stream>>>(c->S.boxes, c->nbox, (uint32_t)n0,
                                                          (uint32_t)count, c->p.grid_shift, c->shifts);
  HIP_TRY(hipGetLastError());
  c->shift_view = c->shifts;
  c->shift_n0 = n0;
  c->shift_count = count;
  return MPCD_OK;
}

const ShiftEntry* shift_at(const mpcd_ctx c, uint64_t n) {
  return c->shift_view + (n - c->shift_n0) * c->nbox;
}

// --- profiling helpers
hipEvent_t pool_event(mpcd_ctx c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  mpcd_ctx c;
  int which;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(mpcd_ctx c_, int w) : c(c_), which(w) {
    if (c->prof_every <= 0) return;
    if (c->prof_seen[which]++ % (uint64_t)c->prof_every != 0) return;
    e0 = pool_event(c);
    e1 = pool_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, c->stream);
  }
  ~ProfScope() {
    if (!e0 || !e1) return;
    (void)hipEventRecord(e1, c->stream);
    c->ev_used[which].emplace_back(e0, e1);
  }
};

uint32_t slab_blocks(const mpcd_ctx c, uint32_t cap) {
  return c->S.ntiles * ((cap + 255u) / 256u);
}

// --- tile kernel dispatch
template <int F, int CPT, int MODE, bool SI, bool AT>
void tile_inst2(mpcd_ctx c, const TileArgs& a, bool th, bool em) {
  const uint32_t nb = c->S.ntiles;
  if constexpr (AT) {  // the AT rule runs without the rotation's thermostat
    if (em) k_tile<F, CPT, MODE, SI, false, true, true><<<nb, TT, 0, c->stream>>>(a);
    else k_tile<F, CPT, MODE, SI, false, false, true><<<nb, TT, 0, c->stream>>>(a);
  } else if (th) {
    if (em) k_tile<F, CPT, MODE, SI, true, true, false><<<nb, TT, 0, c->stream>>>(a);
    else k_tile<F, CPT, MODE, SI, true, false, false><<<nb, TT, 0, c->stream>>>(a);
  } else {
    if (em) k_tile<F, CPT, MODE, SI, false, true, false><<<nb, TT, 0, c->stream>>>(a);
    else k_tile<F, CPT, MODE, SI, false, false, false><<<nb, TT, 0, c->stream>>>(a);
  }
}

template <int F, int CPT>
void tile_inst1(mpcd_ctx c, const TileArgs& a, int mode, bool stream_in, bool th, bool em, bool at) {
  switch (mode) {
    case MODE_BIN:
      // binning needs no cell sums: thermostat/embedded/rule variants are the same
      if (stream_in) tile_inst2<F, CPT, MODE_BIN, true, false>(c, a, false, false);
      else tile_inst2<F, CPT, MODE_BIN, false, false>(c, a, false, false);
      break;
    case MODE_COLLIDE:
      if (at) tile_inst2<F, CPT, MODE_COLLIDE, false, true>(c, a, th, em);
      else tile_inst2<F, CPT, MODE_COLLIDE, false, false>(c, a, th, em);
      break;
    case MODE_COLLIDE_SCATTER:
      if (at) tile_inst2<F, CPT, MODE_COLLIDE_SCATTER, false, true>(c, a, th, em);
      else tile_inst2<F, CPT, MODE_COLLIDE_SCATTER, false, false>(c, a, th, em);
      break;
    default: tile_inst2<F, CPT, MODE_DIAG, false, false>(c, a, th, em); break;  // cell sums only
  }
}

template <int F>
void tile_dispatch(mpcd_ctx c, const TileArgs& a, int mode, bool stream_in) {
  const bool th = c->p.thermostat != 0, em = c->n_emb > 0, at = c->p.collision == MPCD_AT;
  switch (c->cpt) {
    case 64: tile_inst1<F, 64>(c, a, mode, stream_in, th, em, at); break;
    case 128: tile_inst1<F, 128>(c, a, mode, stream_in, th, em, at); break;
    default: tile_inst1<F, 256>(c, a, mode, stream_in, th, em, at); break;
  }
}

TileArgs tile_args(mpcd_ctx c) {
  TileArgs a{};
  a.in = c->buf[c->cur];
  a.out = c->buf[1 - c->cur];
  a.S = c->S;
  a.cnt_in = c->cnt[c->ci];
  a.cnt_out = c->cnt[(c->ci + 1) % 3];
  a.cnt_clear = c->cnt[(c->ci + 2) % 3];
  a.emb_mass = c->emb_mass;
  a.status = c->status;
  a.eslot_out = c->n_emb ? c->eslot[1 - c->cur] : nullptr;
  a.one_box = c->nbox == 1 ? 1u : 0u;
  return a;
}

// One tile-kernel launch for step n. The shift table must hold step n (and
// n + 1 for a collision fused with the next binning).
mpcd_status launch_tile(mpcd_ctx c, Op op, uint64_t n, uint32_t seq) {
  TileArgs a = tile_args(c);
  a.step = (uint32_t)n;
  a.seq = seq;
  a.sh = shift_at(c, n);
  int mode;
  bool stream_in = false;
  switch (op) {
    case Op::BinStream: mode = MODE_BIN; stream_in = true; break;
    case Op::Bin: mode = MODE_BIN; break;
    case Op::CollideScatter: mode = MODE_COLLIDE_SCATTER; a.shn = shift_at(c, n + 1); break;
    case Op::CollideLast:
      mode = MODE_COLLIDE_SCATTER;
      a.shn = shift_at(c, n + 1);
      break;
    default: mode = MODE_COLLIDE; break;
  }
  {
    ProfScope ps(c, mode == MODE_BIN ? 1 : 0);
    if (c->form == 0) tile_dispatch<0>(c, a, mode, stream_in);
    else tile_dispatch<1>(c, a, mode, stream_in);
    HIP_TRY(hipGetLastError());
  }
  if (op == Op::CollideLast) {  // the input stays current; the output is the prepared next binning
    c->pre = true;
    c->split = true;
    return MPCD_OK;
  }
  c->cur = 1 - c->cur;
  if (mode != MODE_COLLIDE) c->ci = (c->ci + 1) % 3;
  return MPCD_OK;
}

// --- slabs
mpcd_status alloc_slabs(mpcd_ctx c, uint32_t cap, Particles out[2], std::vector<void*>& owned) {
  const size_t S = (size_t)c->S.ntiles * cap;
  auto get = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (c->alloc(&q, bytes) != hipSuccess) return nullptr;
    owned.push_back(q);
    return q;
  };
  for (int b = 0; b < 2; ++b) {
    Particles& P = out[b];
    P = Particles{};
    if (c->form == 0) {
      P.wa = (double2*)get(S * 16);
      P.wb = (double2*)get(S * 16);
      P.wc = (double2*)get(S * 16);
      if (!P.wa || !P.wb || !P.wc) return fail(MPCD_ENOMEM, "device allocation of the slabs failed");
      P.tag = (uint32_t*)get(S * 4);
      if (!P.tag) return fail(MPCD_ENOMEM, "device allocation of the slabs failed");
    } else {
      P.ra = (uint4*)get(S * 16);
      P.rb = (uint4*)get(S * 16);
      if (!P.ra || !P.rb) return fail(MPCD_ENOMEM, "device allocation of the slabs failed");
    }
  }
  return MPCD_OK;
}

void free_all(mpcd_ctx c, std::vector<void*>& v) {
  for (void* q : v) c->release(q);
  v.clear();
}

// A slab overflowed in a launch whose input was (in_cur, in_ci). Enlarge
// the slabs to hold the largest count the failed launch tried to place (plus
// headroom), repack that intact input and reset the counters.
mpcd_status regrow(mpcd_ctx c, int in_cur, int in_ci) {
  const uint32_t nt = c->S.ntiles;
  std::vector<uint32_t> want(nt);
  HIP_TRY(hipMemcpy(want.data(), c->cnt[(in_ci + 1) % 3], (size_t)nt * 4, hipMemcpyDeviceToHost));
  uint32_t mx = 0;
  for (uint32_t v : want) mx = std::max(mx, v);
  const uint32_t old_cap = c->S.cap;
  const uint64_t target = std::max<uint64_t>((uint64_t)mx + mx / 4 + 64, (uint64_t)old_cap + old_cap / 2);
  const uint32_t new_cap = round_up(target, 64);
  if ((uint64_t)new_cap * nt >= (1ull << 32) || new_cap >= kMaxCap)
    return fail(MPCD_ENOMEM, "slab storage beyond 2^32 slots or 2^28 per tile");
  Particles nb[2];
  std::vector<void*> owned;
  mpcd_status st = alloc_slabs(c, new_cap, nb, owned);
  if (st != MPCD_OK) {
    free_all(c, owned);
    return st;
  }
  Slabs S = c->S;
  S.cap = new_cap;
  const uint32_t blocks = nt * ((old_cap + 255u) / 256u);
  if (c->form == 0)
    k_repack<0><<<blocks, 256, 0, c->stream>>>(c->buf[in_cur], nb[0], S, old_cap, c->cnt[in_ci],
                                               c->n_emb ? c->eslot[0] : nullptr);
  else
    k_repack<1><<<blocks, 256, 0, c->stream>>>(c->buf[in_cur], nb[0], S, old_cap, c->cnt[in_ci],
                                               c->n_emb ? c->eslot[0] : nullptr);
  HIP_TRY(hipGetLastError());
  if (in_ci != 0)
    HIP_TRY(hipMemcpyAsync(c->cnt[0], c->cnt[in_ci], (size_t)nt * 4, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->cnt[1], 0, (size_t)nt * 4, c->stream));
  HIP_TRY(hipMemsetAsync(c->cnt[2], 0, (size_t)nt * 4, c->stream));
  const uint32_t st_reset[2] = {0u, 0xFFFFFFFFu};
  HIP_TRY(hipMemcpyAsync(c->status + 1, st_reset, 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  free_all(c, c->slab_allocs);
  c->slab_allocs = owned;
  c->buf[0] = nb[0];
  c->buf[1] = nb[1];
  c->S.cap = new_cap;
  c->cur = 0;
  c->ci = 0;
  c->pre = false;
  c->split = false;
  c->regrows += 1;
  return MPCD_OK;
}

// Join a split state in buf[cur]: the velocities of the prepared buffer
// are copied, by tag, into the slots of the current one.
mpcd_status materialize(mpcd_ctx c) {
  if (!c->split) return MPCD_OK;
  c->split = false;
  if (c->N == 0) return MPCD_OK;
  void* tmp = nullptr;
  HIP_TRY(c->alloc(&tmp, (size_t)c->N * 3 * (c->form == 0 ? 8 : 4)));
  const uint32_t nb = slab_blocks(c, c->S.cap);
  const Particles in = c->buf[c->cur], out = c->buf[1 - c->cur];
  const uint32_t *cn_in = c->cnt[c->ci], *cn_out = c->cnt[(c->ci + 1) % 3];
  if (c->form == 0) {
    k_vel_by_tag<0><<<nb, kGrid, 0, c->stream>>>(out, c->S, cn_out, (double*)tmp);
    k_vel_from_tag<0><<<nb, kGrid, 0, c->stream>>>(in, c->S, cn_in, (const double*)tmp);
  } else {
    k_vel_by_tag<1><<<nb, kGrid, 0, c->stream>>>(out, c->S, cn_out, (float*)tmp);
    k_vel_from_tag<1><<<nb, kGrid, 0, c->stream>>>(in, c->S, cn_in, (const float*)tmp);
  }
  const hipError_t e = hipGetLastError();
  c->release(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "materialize: %s", hipGetErrorString(e));
  return MPCD_OK;
}

// Give up the binning prepared by the last mpcd_step (after joining a split
// state). Its counts sit in cnt[(ci + 1) % 3], which the next scatter would
// add to, while the counts the last collide + scatter cleared sit in
// cnt[(ci + 2) % 3]: swapping the two pointers hands the next scatter clean
// counts and leaves the stale ones to be cleared by it.
mpcd_status drop_prepared(mpcd_ctx c) {
  if (!c->pre) return MPCD_OK;
  ST_TRY(materialize(c));
  std::swap(c->cnt[(c->ci + 1) % 3], c->cnt[(c->ci + 2) % 3]);
  c->pre = false;
  return MPCD_OK;
}

// Enqueue launches L[from..] as one graph: capture them on the context's
// stream (thread-local mode: other threads' calls are unaffected), update the
// kept executable graph with the capture, or instantiate a new one when the
// update is refused (another shape), and launch it. in_state records the
// (buffer, counter) pair each launch reads.
mpcd_status launch_graph(mpcd_ctx c, const std::vector<Launch>& L, size_t from,
                         std::vector<std::pair<int, int>>& in_state) {
  HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  mpcd_status st = MPCD_OK;
  for (size_t k = from; k < L.size() && st == MPCD_OK; ++k) {
    in_state.emplace_back(c->cur, c->ci);
    st = launch_tile(c, L[k].op, L[k].step, (uint32_t)(k - from));
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (st != MPCD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(MPCD_EHIP, "graph capture: %s", hipGetErrorString(e));
  bool updated = false;
  if (c->gexec) {
    hipGraphNode_t bad_node = nullptr;
    hipGraphExecUpdateResult res;
    updated = hipGraphExecUpdate(c->gexec, g, &bad_node, &res) == hipSuccess &&
              res == hipGraphExecUpdateSuccess;
    if (!updated) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
  }
  if (!updated) {
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      c->gexec = nullptr;
      (void)hipGraphDestroy(g);
      return fail(MPCD_EHIP, "graph instantiation: %s", hipGetErrorString(ei));
    }
    c->graph_inst += 1;
  } else {
    c->graph_upd += 1;
  }
  const hipError_t el = hipGraphLaunch(c->gexec, c->stream);
  (void)hipGraphDestroy(g);
  if (el != hipSuccess) return fail(MPCD_EHIP, "graph launch: %s", hipGetErrorString(el));
  return MPCD_OK;
}

// A launch overflowed a slab and the slabs could not be enlarged: return to
// that launch's input (cur, ci), which it and every later launch of the call
// left intact, and clear the counts it added to. A stream + bin launch's
// input is the state before the call (or, for mpcd_bin, the streamed
// state); a collision's input is its step binned and not yet collided.
mpcd_status rollback_to_input(mpcd_ctx c, int cur, int ci, const Launch& l) {
  c->cur = cur;
  c->ci = ci;
  c->pre = false;
  c->split = false;
  if (l.op == Op::BinStream) {
    c->phase = Phase::Idle;
  } else if (l.op == Op::Bin) {
    c->phase = Phase::Streamed;
  } else {
    c->phase = Phase::Binned;
    c->step = l.step;
    c->have_bin = true;
    c->last_bin_step = l.step;
  }
  const uint32_t st_reset[2] = {0u, 0xFFFFFFFFu};
  HIP_TRY(hipMemsetAsync(c->cnt[(c->ci + 1) % 3], 0, (size_t)c->S.ntiles * 4, c->stream));
  HIP_TRY(hipMemcpyAsync(c->status + 1, st_reset, 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MPCD_OK;
}

// Run a list of tile launches, then confirm that no slab overflowed; replay
// from the failing launch after enlarging the slabs if one did.
mpcd_status run_launches(mpcd_ctx c, const std::vector<Launch>& L) {
  size_t from = 0;
  for (int attempt = 0; attempt < 16; ++attempt) {
    std::vector<std::pair<int, int>> in_state;
    in_state.reserve(L.size() - from);
    if (c->graph && c->prof_every == 0) {
      ST_TRY(launch_graph(c, L, from, in_state));
    } else {
      for (size_t k = from; k < L.size(); ++k) {
        in_state.emplace_back(c->cur, c->ci);
        ST_TRY(launch_tile(c, L[k].op, L[k].step, (uint32_t)(k - from)));
      }
    }
    uint32_t st[3];
    HIP_TRY(hipMemcpyAsync(st, c->status, 12, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (st[1] == 0) return MPCD_OK;
    const size_t bad = std::min<size_t>(st[2], in_state.size() - 1);
    const mpcd_status rs = regrow(c, in_state[bad].first, in_state[bad].second);
    if (rs != MPCD_OK) {
      const std::string why = g_err;
      ST_TRY(rollback_to_input(c, in_state[bad].first, in_state[bad].second, L[from + bad]));
      return fail(rs, "%s; the state is %s", why.c_str(),
                  c->phase == Phase::Binned ? "the failing step binned, awaiting mpcd_collide"
                  : c->phase == Phase::Streamed ? "streamed, awaiting mpcd_bin"
                                                : "the one before the call");
    }
    from += bad;
  }
  return fail(MPCD_ENOMEM, "slab capacity kept overflowing");
}

int tile_shape(const mpcd_params& p) {
  return (int)(((uint32_t)p.flags & MPCD_TILE_MASK) >> MPCD_TILE_SHIFT);
}

mpcd_status validate(const mpcd_params* p, int64_t ns, int64_t ne) {
  if (!p) return fail(MPCD_EINVAL, "params is NULL");
  for (int d = 0; d < 3; ++d)
    if (p->n_cells[d] < 1) return fail(MPCD_EINVAL, "n_cells[%d] = %d < 1", d, p->n_cells[d]);
  const double nc = (double)p->n_cells[0] * p->n_cells[1] * p->n_cells[2];
  if (nc > 4.0e9) return fail(MPCD_EINVAL, "too many cells (%.0f)", nc);
  if (!(p->a > 0.0) || !std::isfinite(p->a)) return fail(MPCD_EINVAL, "cell size a must be > 0");
  if (!(p->dt >= 0.0) || !std::isfinite(p->dt)) return fail(MPCD_EINVAL, "dt must be >= 0");
  if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return fail(MPCD_EINVAL, "kT must be >= 0");
  if (!std::isfinite(p->alpha)) return fail(MPCD_EINVAL, "alpha must be finite");
  if (!(p->solvent_mass > 0.0) || !std::isfinite(p->solvent_mass))
    return fail(MPCD_EINVAL, "solvent_mass must be > 0");
  if (p->precision != MPCD_FP64 && p->precision != MPCD_FP32)
    return fail(MPCD_EINVAL, "precision must be MPCD_FP64 or MPCD_FP32");
  if (p->thermostat != 0 && p->thermostat != 1) return fail(MPCD_EINVAL, "thermostat must be 0 or 1");
  if (p->grid_shift != 0 && p->grid_shift != 1) return fail(MPCD_EINVAL, "grid_shift must be 0 or 1");
  if ((uint32_t)p->flags & ~(uint32_t)(MPCD_FLAG_TIGHT_SLABS | MPCD_FLAG_MD_SOLUTE | MPCD_TILE_MASK))
    return fail(MPCD_EINVAL, "unknown flags");
  if (tile_shape(*p) > 4) return fail(MPCD_EINVAL, "unknown tile shape %d", tile_shape(*p));
  if (p->collision != MPCD_SRD && p->collision != MPCD_AT)
    return fail(MPCD_EINVAL, "collision must be MPCD_SRD or MPCD_AT");
  if (p->collision == MPCD_AT && p->thermostat)
    return fail(MPCD_EINVAL, "the AT rule thermostats by itself: thermostat must be 0");
  if (p->precision == MPCD_FP32)
    for (int d = 0; d < 3; ++d)
      if (p->n_cells[d] > 1024) return fail(MPCD_EINVAL, "FP32 form supports at most 1024 cells per axis");
  if (ns < 0 || ne < 0) return fail(MPCD_EINVAL, "negative particle count");
  if (ns + ne >= (int64_t)1 << 31) return fail(MPCD_EINVAL, "at most 2^31 - 1 particles");
  return MPCD_OK;
}

// Tile shape of one box by its mean density rho, from step times measured
// for every shape on one MI355X (96^3-cell boxes, both forms, both rules):
//  - a box alone, SRD rule: 8x8x4 cells below 3.75 particles per cell,
//    8x4x4 below 7.5, 4x4x4 below 12, 4x4x2 from 12 (each within 5 % of the
//    fastest shape at the densities measured, 1.5-12 % faster than the
//    shape of the next band);
//  - a box alone, AT rule in the FP64 form: 8x8x4 below 2.5, 4x4x4 below
//    12, 4x4x2 from 12 (its kernels lose more occupancy with larger tiles);
//    the FP32 form's AT kernels follow the SRD rule;
//  - boxes of a batch: every box runs with the kernel of the largest tile
//    any box needs (cells per tile 64/128/256), which slows the boxes with
//    smaller tiles, so a batch keeps 64-cell tiles down to density 3.5
//    (measured on the 256-box batch: 15 % faster than 128-cell tiles for its
//    boxes from density 7 down), 8x4x4 below, 8x8x4 below 1.75, 4x4x2 from
//    12.
// The kernels hold up to 768 particles of a 64-cell tile and 1024 of a
// larger one in registers; more are read again from memory (the shapes that
// overflow them at a density are many times slower). shape 1..4 (the
// MPCD_TILE_* codes) sets the shape instead of the rule. Returns the cells
// per tile, rounded up to the kernel sizes 64/128/256.
int choose_tiles(Box& B, double rho, int shape = 0, bool single = true, bool at_rule = false) {
  if (shape == 0) {
    if (rho >= 12.0) shape = 1;
    else if (!single) shape = rho >= 3.5 ? 2 : (rho >= 1.75 ? 3 : 4);
    else if (at_rule) shape = rho >= 2.5 ? 2 : 4;
    else shape = rho >= 7.5 ? 2 : (rho >= 3.75 ? 3 : 4);
  }
  int td[3], cpt;
  if (shape == 1) {
    td[0] = 4; td[1] = 4; td[2] = 2; cpt = 64;
  } else if (shape == 2) {
    td[0] = 4; td[1] = 4; td[2] = 4; cpt = 64;
  } else if (shape == 3) {
    td[0] = 8; td[1] = 4; td[2] = 4; cpt = 128;
  } else {
    td[0] = 8; td[1] = 8; td[2] = 4; cpt = 256;
  }
  B.ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    if (B.n[d] <= td[d]) {
      B.td[d] = B.n[d];
      B.nt[d] = 1;
      B.tsh[d] = 31;  // every cell coordinate (< 2^10) shifts to tile 0
      B.lm[d] = 0xFFFFFFFFu;
    } else {
      B.td[d] = td[d];
      B.nt[d] = (B.n[d] + td[d] - 1) / td[d];
      int sh = 0;
      while ((1 << sh) < td[d]) ++sh;
      B.tsh[d] = sh;
      B.lm[d] = (uint32_t)td[d] - 1u;
    }
    B.ntiles *= (uint32_t)B.nt[d];
  }
  B.m_td0 = (uint32_t)(((1u << 24) + B.td[0] - 1) / B.td[0]);
  B.m_td01 = (uint32_t)(((1u << 24) + B.td[0] * B.td[1] - 1) / (B.td[0] * B.td[1]));
  B.inv_nt0 = 1.0 / (double)B.nt[0];
  B.inv_nt01 = 1.0 / ((double)B.nt[0] * (double)B.nt[1]);
  return cpt;
}

// Slots per tile slab: 1.2 x the largest initial tile occupancy, and at least
// the mean occupancy plus eight standard deviations (Poisson) plus 64,
// rounded up to 32.
uint32_t slab_cap(uint64_t max_occupancy, double mean) {
  const uint64_t want = std::max<uint64_t>(max_occupancy + max_occupancy / 5,
                                           (uint64_t)(mean + 8.0 * std::sqrt(mean) + 64.0));
  return round_up(want, 32);
}

// Per-box constants from the parameters (layout fields are set by the caller).
Box make_box(const mpcd_params& p) {
  Box B{};
  for (int d = 0; d < 3; ++d) {
    B.n[d] = p.n_cells[d];
    B.L[d] = (double)p.n_cells[d] * p.a;
  }
  B.a = p.a;
  B.inv_a = 1.0 / p.a;
  B.dt = p.dt;
  B.a32 = (float)p.a;
  B.inv_a32 = (float)B.inv_a;
  B.dt32 = (float)p.dt;
  B.ncells = (uint32_t)((uint64_t)p.n_cells[0] * p.n_cells[1] * p.n_cells[2]);
  B.ca = std::cos(p.alpha);
  B.sa = std::sin(p.alpha);
  B.omc = 1.0 - B.ca;
  B.kT = p.kT;
  B.mass = p.solvent_mass;
  B.k0 = (uint32_t)(p.seed & 0xFFFFFFFFull);
  B.k1 = (uint32_t)(p.seed >> 32);
  B.md_solute = ((uint32_t)p.flags & MPCD_FLAG_MD_SOLUTE) ? 1u : 0u;
  return B;
}

// Create a context of nbox boxes. Box b has n_solv[b] solvent particles,
// rows [row0_b, row0_b + n_solv[b]) of pos/vel (row0 = running sum); box 0
// may also have n_emb embedded particles.
mpcd_status create_impl(int32_t nbox, const mpcd_params* params, const int64_t* n_solv,
                        const double* pos, const double* vel, int64_t n_embedded,
                        const double* emb_pos, const double* emb_vel, const double* emb_mass,
                        int32_t pointers_on_device, void* hip_stream, mpcd_ctx* out) {
  g_err.clear();
  if (!out) return fail(MPCD_EINVAL, "out is NULL");
  *out = nullptr;
  if (nbox < 1) return fail(MPCD_EINVAL, "n_boxes must be >= 1");
  if (!params || !n_solv) return fail(MPCD_EINVAL, "params/n_particles is NULL");
  int64_t ns_total = 0;
  double ncells_total = 0.0;
  for (int32_t b = 0; b < nbox; ++b) {
    mpcd_status st = validate(&params[b], n_solv[b], b == 0 ? n_embedded : 0);
    if (st != MPCD_OK) {
      if (nbox > 1) g_err = "box " + std::to_string(b) + ": " + g_err;
      return st;
    }
    const mpcd_params& q = params[b];
    if (q.precision != params[0].precision || q.thermostat != params[0].thermostat ||
        q.grid_shift != params[0].grid_shift ||
        ((q.flags ^ params[0].flags) & ~(int32_t)MPCD_TILE_MASK) != 0 ||
        q.collision != params[0].collision)
      return fail(MPCD_EINVAL,
                  "box %d: precision, thermostat, grid_shift, flags (but the tile shape) and "
                  "collision must match box 0", b);
    ns_total += n_solv[b];
    ncells_total += (double)q.n_cells[0] * q.n_cells[1] * q.n_cells[2];
  }
  if (ns_total + n_embedded >= (int64_t)1 << 31) return fail(MPCD_EINVAL, "at most 2^31 - 1 particles");
  if (ncells_total > 4.0e9) return fail(MPCD_EINVAL, "too many cells (%.0f)", ncells_total);
  if (ns_total > 0 && (!pos || !vel)) return fail(MPCD_EINVAL, "pos/vel NULL");
  if (n_embedded > 0 && (!emb_pos || !emb_vel || !emb_mass))
    return fail(MPCD_EINVAL, "embedded arrays NULL");
  if (n_embedded > 0 && !pointers_on_device) {
    for (int64_t i = 0; i < n_embedded; ++i)
      if (!(emb_mass[i] > 0.0) || !std::isfinite(emb_mass[i]))
        return fail(MPCD_EINVAL, "embedded mass %lld is not > 0", (long long)i);
  }

  mpcd_ctx c = new (std::nothrow) mpcd_ctx_s();
  if (!c) return fail(MPCD_ENOMEM, "host allocation failed");
  auto cleanup = [&](mpcd_status s) {
    std::string keep = g_err;
    mpcd_destroy(c);
    g_err = keep;
    return s;
  };
  c->p = params[0];
  c->form = params[0].precision;
  c->nbox = (uint32_t)nbox;
  c->n_emb = (uint32_t)n_embedded;
  c->N = (uint32_t)(ns_total + n_embedded);

  // boxes and the tile layout
  uint32_t tile = 0, tag = 0;
  uint64_t cell = 0;
  int cpt = 64;
  std::vector<uint32_t> tile_box;
  double max_mean = 0.0;
  for (int32_t b = 0; b < nbox; ++b) {
    Box B = make_box(params[b]);
    const uint32_t nb = (uint32_t)n_solv[b] + (b == 0 ? c->n_emb : 0u);
    cpt = std::max(cpt, choose_tiles(B, B.ncells ? (double)nb / (double)B.ncells : 0.0,
                                     tile_shape(params[b]), nbox == 1,
                                     params[b].collision == MPCD_AT &&
                                         params[b].precision == MPCD_FP64));
    const uint32_t t0 = tile;
    B.tile0 = t0;
    B.tag0 = tag;
    B.cell0 = (uint32_t)cell;
    B.n_solvent = (uint32_t)n_solv[b];
    tile_box.resize(t0 + B.ntiles, (uint32_t)b);
    max_mean = std::max(max_mean, (double)nb / (double)B.ntiles);
    tile = t0 + B.ntiles;
    tag += nb;
    cell += B.ncells;
    c->boxes.push_back(B);
    c->box_n.push_back(nb);
  }
  const uint32_t NT = tile;
  c->cpt = cpt;
  c->ncells = cell;
  c->S.ntiles = NT;

  if (hipGetDevice(&c->device) != hipSuccess)
    return cleanup(fail(MPCD_EHIP, "hipGetDevice failed (no usable GPU?)"));
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return cleanup(fail(MPCD_EHIP, "hipStreamCreate failed (no usable GPU?)"));
    c->own_stream = true;
  }
  for (int k = 0; k < 3; ++k) c->cnt[k] = (uint32_t*)c->dalloc((size_t)NT * 4);
  c->status = (uint32_t*)c->dalloc(256);
  c->tot = (long long*)c->dalloc((size_t)nbox * 10 * 8);
  c->emb_mass = (double*)c->dalloc((size_t)c->n_emb * 8);
  Box* dboxes = (Box*)c->dalloc((size_t)nbox * sizeof(Box));
  uint32_t* dtb = (uint32_t*)c->dalloc((size_t)NT * 4);
  uint32_t* bad = (uint32_t*)c->dalloc(256);
  c->flag = bad;
  if (c->n_emb) {
    c->eslot[0] = (uint32_t*)c->dalloc((size_t)c->n_emb * 4);
    c->eslot[1] = (uint32_t*)c->dalloc((size_t)c->n_emb * 4);
    if (!c->eslot[0] || !c->eslot[1]) return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
  }
  if (!c->cnt[0] || !c->cnt[1] || !c->cnt[2] || !c->status || !c->tot || !c->emb_mass || !dboxes ||
      !dtb || !bad)
    return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
  c->S.boxes = dboxes;
  c->S.tile_box = dtb;
  const uint32_t st_init[8] = {0u, 0u, 0xFFFFFFFFu, 0u, 0u, 0u, 0u, 0u};
  if (hipMemsetAsync(c->cnt[0], 0, (size_t)NT * 4, c->stream) != hipSuccess ||
      hipMemsetAsync(c->cnt[1], 0, (size_t)NT * 4, c->stream) != hipSuccess ||
      hipMemsetAsync(c->cnt[2], 0, (size_t)NT * 4, c->stream) != hipSuccess ||
      hipMemsetAsync(bad, 0, 256, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->status, st_init, sizeof st_init, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(dboxes, c->boxes.data(), (size_t)nbox * sizeof(Box), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess ||
      hipMemcpyAsync(dtb, tile_box.data(), (size_t)NT * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return cleanup(fail(MPCD_EHIP, "create: upload of the layout failed"));

  // upload: host arrays are staged through temporary device buffers
  struct Src {
    const double* p;
    const double* v;
    uint64_t n;
    double* tmp;
  } src[2] = {{pos, vel, (uint64_t)ns_total, nullptr}, {emb_pos, emb_vel, c->n_emb, nullptr}};
  auto free_tmp = [&]() {
    for (auto& s : src)
      if (s.tmp) {
        c->release(s.tmp);
        s.tmp = nullptr;
      }
  };
  for (auto& s : src) {
    if (s.n == 0 || pointers_on_device) continue;
    if (c->alloc((void**)&s.tmp, (size_t)s.n * 48) != hipSuccess) {
      free_tmp();
      return cleanup(fail(MPCD_ENOMEM, "device allocation of the upload buffer failed"));
    }
    if (hipMemcpyAsync(s.tmp, s.p, (size_t)s.n * 24, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(s.tmp + 3 * (size_t)s.n, s.v, (size_t)s.n * 24, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      free_tmp();
      return cleanup(fail(MPCD_EHIP, "upload failed"));
    }
    s.p = s.tmp;
    s.v = s.tmp + 3 * (size_t)s.n;
  }
  // one import launch per (box, particle kind)
  auto import_all = [&](bool place, uint32_t cap, uint32_t* cnt) {
    uint32_t* es = c->n_emb ? c->eslot[0] : nullptr;
    uint64_t row = 0;
    for (uint32_t b = 0; b < c->nbox; ++b) {
      const Box& B = c->boxes[b];
      struct Part {
        const double* p;
        const double* v;
        uint32_t n, tag0;
      } parts[2] = {{src[0].p + 3 * row, src[0].v + 3 * row, B.n_solvent, B.tag0},
                    {src[1].p, src[1].v, b == 0 ? c->n_emb : 0u, B.tag0 + B.n_solvent}};
      row += B.n_solvent;
      for (const Part& q : parts) {
        if (q.n == 0) continue;
        const uint32_t g = blocks_for(q.n, kGrid);
        if (c->form == 0) {
          if (place) k_import<0, true><<<g, kGrid, 0, c->stream>>>(c->buf[0], B, cap, q.p, q.v, q.n, q.tag0, cnt, bad, es);
          else k_import<0, false><<<g, kGrid, 0, c->stream>>>(c->buf[0], B, cap, q.p, q.v, q.n, q.tag0, cnt, bad, es);
        } else {
          if (place) k_import<1, true><<<g, kGrid, 0, c->stream>>>(c->buf[0], B, cap, q.p, q.v, q.n, q.tag0, cnt, bad, es);
          else k_import<1, false><<<g, kGrid, 0, c->stream>>>(c->buf[0], B, cap, q.p, q.v, q.n, q.tag0, cnt, bad, es);
        }
      }
    }
  };
  // pass 1: count per tile, check the box
  import_all(false, 0u, c->cnt[1]);
  std::vector<uint32_t> cnt_h(NT);
  uint32_t hbad = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(cnt_h.data(), c->cnt[1], (size_t)NT * 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    free_tmp();
    return cleanup(fail(MPCD_EHIP, "create: import failed"));
  }
  if (hbad) {
    free_tmp();
    return cleanup(fail(MPCD_EINVAL, "a position lies outside [0, L)"));
  }
  uint32_t mx = 0;
  for (uint32_t v : cnt_h) mx = std::max(mx, v);
  uint32_t cap;
  if ((uint32_t)params[0].flags & MPCD_FLAG_TIGHT_SLABS) {
    cap = std::max<uint32_t>(mx, 1u);
  } else {
    cap = slab_cap(mx, max_mean);
  }
  if ((uint64_t)cap * NT >= (1ull << 32) || cap >= kMaxCap) {
    free_tmp();
    return cleanup(fail(MPCD_ENOMEM, "slab storage beyond 2^32 slots or 2^28 per tile"));
  }
  c->S.cap = cap;
  mpcd_status st = alloc_slabs(c, cap, c->buf, c->slab_allocs);
  if (st != MPCD_OK) {
    free_tmp();
    return cleanup(st);
  }
  if (hipMemsetAsync(c->cnt[1], 0, (size_t)NT * 4, c->stream) != hipSuccess) {
    free_tmp();
    return cleanup(fail(MPCD_EHIP, "hipMemset failed"));
  }
  // pass 2: place
  import_all(true, cap, c->cnt[0]);
  if (c->n_emb) {
    if (hipMemcpyAsync(c->emb_mass, emb_mass, (size_t)c->n_emb * 8,
                       pointers_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
      free_tmp();
      return cleanup(fail(MPCD_EHIP, "upload of embedded masses failed"));
    }
  }
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    free_tmp();
    return cleanup(fail(MPCD_EHIP, "create: placement failed"));
  }
  free_tmp();
  if (hbad) return cleanup(fail(MPCD_EHIP, "create: placement exceeded the slab capacity"));
  c->cur = 0;
  c->ci = 0;
  c->step = 0;
  c->phase = Phase::Idle;
  *out = c;
  return MPCD_OK;
}

// Totals of the boxes [b0, b1) from the fixed-point words (integer sums, so
// exact and independent of the order of the boxes).
void totals_of(const mpcd_ctx c, const std::vector<long long>& h, uint32_t b0, uint32_t b1,
               double p[3], double* ke, double* kT) {
  long long w[10] = {0};
  uint64_t n = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    for (int q = 0; q < 10; ++q) w[q] += h[10 * b + q];
    n += c->box_n[b];
  }
  auto val = [&](int q) { return (double)w[2 * q] * 0x1p-20 + (double)w[2 * q + 1] * 0x1p-72; };
  const double P0 = val(0), P1 = val(1), P2 = val(2), K = 0.5 * val(3), M = val(4);
  if (p) {
    p[0] = P0;
    p[1] = P1;
    p[2] = P2;
  }
  if (ke) *ke = K;
  if (kT) *kT = (n > 1 && M > 0) ? 2.0 * (K - 0.5 * (P0 * P0 + P1 * P1 + P2 * P2) / M) / (3.0 * (double)(n - 1)) : 0.0;
}

mpcd_status read_totals(mpcd_ctx c, std::vector<long long>& h) {
  h.assign((size_t)c->nbox * 10, 0);
  if (!c->N) return MPCD_OK;
  HIP_TRY(hipMemsetAsync(c->tot, 0, (size_t)c->nbox * 80, c->stream));
  const uint32_t nb = slab_blocks(c, c->S.cap);
  const bool em = c->n_emb > 0;
  // sums of velocities and masses: the prepared buffer holds them when the
  // state is split
  const Particles P = c->split ? c->buf[1 - c->cur] : c->buf[c->cur];
  const uint32_t* cn = c->split ? c->cnt[(c->ci + 1) % 3] : c->cnt[c->ci];
  if (c->form == 0) {
    if (em) k_totals<0, true><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, c->tot, c->status);
    else k_totals<0, false><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, c->tot, c->status);
  } else {
    if (em) k_totals<1, true><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, c->tot, c->status);
    else k_totals<1, false><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, c->tot, c->status);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h.data(), c->tot, (size_t)c->nbox * 80, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MPCD_OK;
}

// ------------------------------------------- allocation-free stepping
// mpcd_step_noalloc stages the grid shifts of its call in this library-wide
// table instead of the context's own (which mpcd_step allocates on demand).
// Every device the library runs on holds its own copy until the process
// ends; host code reaches a copy through the device address that
// hipGetSymbolAddress returns on that device, never through the name.
static_assert(sizeof(ShiftEntry) == 40, "the header states 40 bytes per grid-shift entry");
static __device__ __align__(256) ShiftEntry scratch[MPCD_NOALLOC_MAX_SHIFTS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
ShiftEntry* g_scratch_ptr[kMaxDevices] = {};  // per device: scratch's device address

// The address of scratch on device dev, which must be current: looked up on
// the first call on that device, kept after.
mpcd_status scratch_on(int dev, ShiftEntry** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MPCD_EHIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !q)
      return fail(MPCD_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<ShiftEntry*>(q);
  }
  *out = g_scratch_ptr[dev];
  return MPCD_OK;
}

// Makes `dev` the current device for a scope and restores the caller's.
struct DeviceScope {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceScope(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceScope() {
    int now = -1;
    if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* mpcd_last_error(void) { return g_err.c_str(); }

mpcd_status mpcd_create(const mpcd_params* params, int64_t n_solvent, const double* pos,
                        const double* vel, int64_t n_embedded, const double* emb_pos,
                        const double* emb_vel, const double* emb_mass,
                        int32_t pointers_on_device, void* hip_stream, mpcd_ctx* out) {
  if (n_solvent < 0 || n_embedded < 0) {
    g_err.clear();
    if (out) *out = nullptr;
    return fail(MPCD_EINVAL, "negative particle count");
  }
  return create_impl(1, params, &n_solvent, pos, vel, n_embedded, emb_pos, emb_vel, emb_mass,
                     pointers_on_device, hip_stream, out);
}

mpcd_status mpcd_create_batch(int32_t n_boxes, const mpcd_params* params,
                              const int64_t* n_particles, const double* pos, const double* vel,
                              int32_t pointers_on_device, void* hip_stream, mpcd_ctx* out) {
  return create_impl(n_boxes, params, n_particles, pos, vel, 0, nullptr, nullptr, nullptr,
                     pointers_on_device, hip_stream, out);
}

void mpcd_destroy(mpcd_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c, c->allocs);
  free_all(c, c->slab_allocs);
  c->release(c->shifts);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& v : c->ev_used)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

mpcd_status mpcd_stream(mpcd_ctx c) {
  ST_TRY(check_ctx(c));
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_stream: expected the state after create or collide");
  ST_TRY(drop_prepared(c));  // the binning that follows overwrites the prepared one
  if (c->N) {
    ProfScope ps(c, 1);
    const uint32_t nb = slab_blocks(c, c->S.cap);
    if (c->form == 0) k_stream<0><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->S, c->cnt[c->ci], c->status);
    else k_stream<1><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->S, c->cnt[c->ci], c->status);
    HIP_TRY(hipGetLastError());
  }
  c->phase = Phase::Streamed;
  return MPCD_OK;
}

mpcd_status mpcd_bin(mpcd_ctx c) {
  ST_TRY(check_ctx(c));
  if (c->phase != Phase::Streamed) return fail(MPCD_ESTATE, "mpcd_bin: expected a preceding mpcd_stream");
  if (c->step >= 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  ST_TRY(ensure_shifts(c, c->step, 1));
  ST_TRY(run_launches(c, {Launch{Op::Bin, c->step}}));
  c->phase = Phase::Binned;
  c->have_bin = true;
  c->last_bin_step = c->step;
  return MPCD_OK;
}

mpcd_status mpcd_collide(mpcd_ctx c) {
  ST_TRY(check_ctx(c));
  if (c->phase != Phase::Binned) return fail(MPCD_ESTATE, "mpcd_collide: expected a preceding mpcd_bin");
  ST_TRY(ensure_shifts(c, c->step, 1));
  ST_TRY(launch_tile(c, Op::Collide, c->step, 0));
  c->step += 1;
  c->phase = Phase::Idle;
  return MPCD_OK;
}

mpcd_status mpcd_step(mpcd_ctx c, int64_t nsteps) {
  ST_TRY(check_ctx(c));
  if (nsteps < 0) return fail(MPCD_EINVAL, "nsteps < 0");
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_step: expected the state after create or collide");
  if (nsteps == 0) return MPCD_OK;
  if (c->step + (uint64_t)nsteps > 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  ST_TRY(ensure_shifts(c, c->step, (uint64_t)nsteps + 1));
  std::vector<Launch> L;
  L.reserve((size_t)nsteps + 1);
  if (c->pre) {  // the last call left this step's binning ready
    c->cur = 1 - c->cur;
    c->ci = (c->ci + 1) % 3;
    c->pre = false;
    c->split = false;
  } else {
    L.push_back({Op::BinStream, c->step});
  }
  for (int64_t k = 0; k < nsteps; ++k) {
    L.push_back({k + 1 < nsteps ? Op::CollideScatter : Op::CollideLast, c->step + (uint64_t)k});
  }
  ST_TRY(run_launches(c, L));
  c->step += (uint64_t)nsteps;
  c->last_bin_step = c->step - 1;
  c->have_bin = true;
  c->phase = Phase::Idle;
  return MPCD_OK;
}

mpcd_status mpcd_step_noalloc(mpcd_ctx c, int64_t nsteps) {
  ST_TRY(check_ctx(c));
  if (nsteps < 0) return fail(MPCD_EINVAL, "nsteps < 0");
  if (c->phase != Phase::Idle)
    return fail(MPCD_ESTATE, "mpcd_step_noalloc: expected the state after create or collide");
  if (nsteps == 0) return MPCD_OK;
  if (c->step + (uint64_t)nsteps > 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  const uint64_t nshift = ((uint64_t)nsteps + 1) * c->nbox;
  if (nshift > (uint64_t)MPCD_NOALLOC_MAX_SHIFTS)
    return fail(MPCD_EINVAL,
                "mpcd_step_noalloc: (nsteps + 1) x n_boxes = %llu grid shifts exceed its table of %d",
                (unsigned long long)nshift, MPCD_NOALLOC_MAX_SHIFTS);
  DeviceScope dev(c->device);
  if (dev.err != hipSuccess) return fail(MPCD_EHIP, "selecting the context's device: %s", hipGetErrorString(dev.err));
  ShiftEntry* table = nullptr;
  ST_TRY(scratch_on(c->device, &table));
  const uint64_t step0 = c->step;
  k_shifts<<<blocks_for(nshift, 256), 256, 0, c->stream>>>(c->S.boxes, c->nbox, (uint32_t)step0,
                                                           (uint32_t)nsteps + 1u, c->p.grid_shift, table);
  HIP_TRY(hipGetLastError());
  c->shift_view = table;
  c->shift_n0 = step0;
  c->shift_count = (uint64_t)nsteps + 1;

  // the launches of mpcd_step (kernel timing off: it would create events)
  const int cur0 = c->cur, ci0 = c->ci;
  const bool adopt = c->pre;
  const int32_t prof = c->prof_every;
  c->prof_every = 0;
  mpcd_status st = MPCD_OK;
  uint32_t seq = 0;
  if (adopt) {  // the last call left this step's binning ready
    c->cur = 1 - c->cur;
    c->ci = (c->ci + 1) % 3;
    c->pre = false;
    c->split = false;
  } else {
    st = launch_tile(c, Op::BinStream, step0, seq++);
  }
  for (int64_t k = 0; k < nsteps && st == MPCD_OK; ++k)
    st = launch_tile(c, k + 1 < nsteps ? Op::CollideScatter : Op::CollideLast, step0 + (uint64_t)k, seq++);
  c->prof_every = prof;
  if (st != MPCD_OK) return st;
  uint32_t h[3];
  HIP_TRY(hipMemcpyAsync(h, c->status, 12, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (h[1] == 0) {
    c->step = step0 + (uint64_t)nsteps;
    c->last_bin_step = c->step - 1;
    c->have_bin = true;
    c->phase = Phase::Idle;
    return MPCD_OK;
  }
  // A slab overflowed in launch h[2]; enlarging the slabs would allocate.
  // Later launches of the call left everything alone and the failing one's
  // input is intact: roll back to that input -- the state before the call if
  // it was the first stream + bin, else step s binned and not yet collided --
  // and clear the counts the failing launch added to.
  const uint32_t bad = std::min<uint32_t>(h[2], seq - 1u);
  c->pre = false;
  c->split = false;
  if (!adopt && bad == 0) {
    c->cur = cur0;
    c->ci = ci0;
    c->phase = Phase::Idle;
  } else {
    const uint64_t k = bad - (adopt ? 0u : 1u);
    c->cur = (cur0 ^ 1) ^ (int)(k & 1u);
    c->ci = (int)((ci0 + 1 + k) % 3);
    c->step = step0 + k;
    c->phase = Phase::Binned;
    c->have_bin = true;
    c->last_bin_step = c->step;
  }
  const uint32_t st_reset[2] = {0u, 0xFFFFFFFFu};
  HIP_TRY(hipMemsetAsync(c->cnt[(c->ci + 1) % 3], 0, (size_t)c->S.ntiles * 4, c->stream));
  HIP_TRY(hipMemcpyAsync(c->status + 1, st_reset, 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return fail(MPCD_ENOMEM,
              "mpcd_step_noalloc: a particle slab is full at step %llu and enlarging it would "
              "allocate; the state is %s (mpcd_step enlarges the slabs)",
              (unsigned long long)(step0 + (adopt ? bad : (bad ? bad - 1u : 0u))),
              c->phase == Phase::Binned ? "that step binned, awaiting mpcd_collide"
                                        : "the one before the call");
}

mpcd_status mpcd_get_state(mpcd_ctx c, double* pos, double* vel, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (!pos || !vel) return fail(MPCD_EINVAL, "pos/vel NULL");
  if (c->N == 0) return take_err(c);
  double* dp = pos;
  double* dv = vel;
  double* tmp = nullptr;
  if (!on_device) {
    HIP_TRY(c->alloc((void**)&tmp, (size_t)c->N * 48));
    dp = tmp;
    dv = tmp + 3 * (size_t)c->N;
  }
  const uint32_t nb = slab_blocks(c, c->S.cap);
  // a split state: positions from the current buffer, velocities from the
  // prepared one
  double* dv_cur = c->split ? nullptr : dv;
  if (c->form == 0)
    k_export<0><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->S, c->cnt[c->ci], dp, dv_cur);
  else
    k_export<1><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->S, c->cnt[c->ci], dp, dv_cur);
  if (c->split) {
    const uint32_t* cn = c->cnt[(c->ci + 1) % 3];
    if (c->form == 0) k_export<0><<<nb, kGrid, 0, c->stream>>>(c->buf[1 - c->cur], c->S, cn, nullptr, dv);
    else k_export<1><<<nb, kGrid, 0, c->stream>>>(c->buf[1 - c->cur], c->S, cn, nullptr, dv);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && tmp) {
    e = hipMemcpyAsync(pos, dp, (size_t)c->N * 24, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(vel, dv, (size_t)c->N * 24, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) c->release(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "get_state: %s", hipGetErrorString(e));
  return take_err(c);
}

mpcd_status mpcd_get_embedded(mpcd_ctx c, double* pos, double* vel, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (c->n_emb == 0) return fail(MPCD_EINVAL, "no embedded particles");
  if (!pos || !vel) return fail(MPCD_EINVAL, "pos/vel NULL");
  const size_t n = c->n_emb;
  double* dp = pos;
  double* dv = vel;
  double* tmp = nullptr;
  if (!on_device) {
    HIP_TRY(c->alloc((void**)&tmp, n * 48));
    dp = tmp;
    dv = tmp + 3 * n;
  }
  const uint32_t nb = blocks_for(n, kGrid);
  hipError_t e = hipMemsetAsync(c->flag, 0, 4, c->stream);
  if (e == hipSuccess) {
    // a split state: positions from the current buffer, velocities from the
    // prepared one, each through its own slot index (one pass)
    const size_t ns = (size_t)c->S.ntiles * c->S.cap;
    const int cb = c->cur, pb = 1 - c->cur;
    if (c->split) {
      if (c->form == 0)
        k_emb_export_split<0><<<nb, kGrid, 0, c->stream>>>(c->buf[cb], c->buf[pb], c->boxes[0], c->eslot[cb], c->eslot[pb], (uint32_t)n, ns, dp, dv, c->flag);
      else
        k_emb_export_split<1><<<nb, kGrid, 0, c->stream>>>(c->buf[cb], c->buf[pb], c->boxes[0], c->eslot[cb], c->eslot[pb], (uint32_t)n, ns, dp, dv, c->flag);
    } else {
      if (c->form == 0)
        k_emb_export<0><<<nb, kGrid, 0, c->stream>>>(c->buf[cb], c->boxes[0], c->eslot[cb], (uint32_t)n, ns, dp, dv, c->flag);
      else
        k_emb_export<1><<<nb, kGrid, 0, c->stream>>>(c->buf[cb], c->boxes[0], c->eslot[cb], (uint32_t)n, ns, dp, dv, c->flag);
    }
    e = hipGetLastError();
  }
  uint32_t hflag = 0;
  if (e == hipSuccess && tmp) {
    e = hipMemcpyAsync(pos, dp, n * 24, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(vel, dv, n * 24, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, c->flag, 4, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) c->release(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "get_embedded: %s", hipGetErrorString(e));
  if (hflag) return fail(MPCD_EHIP, "get_embedded: the embedded-particle index is out of date");
  return take_err(c);
}

// The embedded particles' new state into the current buffer, in place; the
// next step bins them.
hipError_t emb_import(mpcd_ctx c, const double* dp, const double* dv) {
  const uint32_t n = c->n_emb, nb = blocks_for(n, kGrid);
  const size_t ns = (size_t)c->S.ntiles * c->S.cap;
  if (c->form == 0)
    k_emb_import<0><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->boxes[0], c->eslot[c->cur], n, ns, dp, dv, c->flag);
  else
    k_emb_import<1><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->boxes[0], c->eslot[c->cur], n, ns, dp, dv, c->flag);
  return hipGetLastError();
}

// Solutes of an MD integrator handed over while the next step's binning is
// prepared: the new state goes into the current buffer in place and into
// the prepared binning at the cell the prepared step's shift puts it in
// (k_emb_rebin / k_emb_depart / k_emb_arrive), so the solvent's binning is
// kept. When a destination slab is full the prepared binning is given up
// and the state imported as without one. *hflag receives the kernels' flag.
mpcd_status emb_handover(mpcd_ctx c, const double* dp, const double* dv, uint32_t* hflag) {
  const uint32_t n = c->n_emb, nb = blocks_for(n, kGrid);
  const uint32_t nt = c->S.ntiles;
  if (!c->dep_head) {  // all four arrays, or none
    void* q[4] = {nullptr, nullptr, nullptr, nullptr};
    const size_t bytes[4] = {(size_t)nt * 4, (size_t)n * 4, (size_t)n * 4, 256};
    for (int k = 0; k < 4; ++k)
      if (c->alloc(&q[k], bytes[k]) != hipSuccess) {
        for (int j = 0; j < k; ++j) c->release(q[j]);
        return fail(MPCD_ENOMEM, "device allocation for the solute handover failed");
      }
    for (void* p : q) c->allocs.push_back(p);  // owned by the context from here
    HIP_TRY(hipMemsetAsync(q[0], 0xFF, bytes[0], c->stream));
    c->dep_head = (int32_t*)q[0];
    c->dep_next = (int32_t*)q[1];
    c->movers = (uint32_t*)q[2];
    c->nmovers = (uint32_t*)q[3];
  }
  ST_TRY(ensure_shifts(c, c->step, 1));
  const ShiftEntry* sh = shift_at(c, c->step);
  const int pb = 1 - c->cur;
  uint32_t* cnt_p = c->cnt[(c->ci + 1) % 3];
  const size_t ns = (size_t)nt * c->S.cap;
  const uint32_t cap = c->S.cap;
  const Box& B = c->boxes[0];
  HIP_TRY(hipMemsetAsync(c->nmovers, 0, 4, c->stream));
  if (c->form == 0) {
    k_emb_rebin<0><<<nb, kGrid, 0, c->stream>>>(c->buf[pb], c->buf[c->cur], B, sh, c->eslot[pb], c->eslot[c->cur], n, ns, cap, dp, dv, c->dep_head, c->dep_next, c->movers, c->nmovers, c->flag);
    k_emb_depart<0><<<nb, kGrid, 0, c->stream>>>(c->buf[pb], B, c->eslot[pb], cap, cnt_p, c->movers, c->nmovers, c->dep_head, c->dep_next);
    k_emb_arrive<0><<<nb, kGrid, 0, c->stream>>>(c->buf[pb], B, sh, c->eslot[pb], cap, cnt_p, c->movers, c->nmovers, dp, dv, c->flag);
  } else {
    k_emb_rebin<1><<<nb, kGrid, 0, c->stream>>>(c->buf[pb], c->buf[c->cur], B, sh, c->eslot[pb], c->eslot[c->cur], n, ns, cap, dp, dv, c->dep_head, c->dep_next, c->movers, c->nmovers, c->flag);
    k_emb_depart<1><<<nb, kGrid, 0, c->stream>>>(c->buf[pb], B, c->eslot[pb], cap, cnt_p, c->movers, c->nmovers, c->dep_head, c->dep_next);
    k_emb_arrive<1><<<nb, kGrid, 0, c->stream>>>(c->buf[pb], B, sh, c->eslot[pb], cap, cnt_p, c->movers, c->nmovers, dp, dv, c->flag);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(hflag, c->flag, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (!(*hflag & 8u)) {
    c->handovers[0] += 1;
    return MPCD_OK;
  }
  // a destination slab was full: give the prepared binning up (joining the
  // velocities by tag; the movers left out of it are then imported anew)
  c->handovers[1] += 1;
  ST_TRY(drop_prepared(c));
  HIP_TRY(hipMemsetAsync(c->flag, 0, 4, c->stream));
  HIP_TRY(emb_import(c, dp, dv));
  HIP_TRY(hipMemcpyAsync(hflag, c->flag, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return MPCD_OK;
}

mpcd_status mpcd_set_embedded(mpcd_ctx c, const double* pos, const double* vel, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (c->n_emb == 0) return fail(MPCD_EINVAL, "no embedded particles");
  if (!pos || !vel) return fail(MPCD_EINVAL, "pos/vel NULL");
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_set_embedded: only between steps");
  // solutes of an MD integrator are not streamed: with the next step's
  // binning prepared they are moved into it; otherwise the next step bins
  // them afresh
  const bool handover = c->pre && (c->p.flags & MPCD_FLAG_MD_SOLUTE);
  if (!handover) ST_TRY(drop_prepared(c));
  const size_t n = c->n_emb;
  const double* dp = pos;
  const double* dv = vel;
  double* tmp = nullptr;  // host arrays are staged through device memory
  hipError_t e = hipSuccess;
  if (!on_device) {
    HIP_TRY(c->alloc((void**)&tmp, n * 48));
    e = hipMemcpyAsync(tmp, pos, n * 24, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(tmp + 3 * n, vel, n * 24, hipMemcpyHostToDevice, c->stream);
    dp = tmp;
    dv = tmp + 3 * n;
  }
  if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, 4, c->stream);
  uint32_t hbad = 0;
  if (handover) {
    if (e == hipSuccess) {
      const mpcd_status st = emb_handover(c, dp, dv, &hbad);
      if (st != MPCD_OK) {
        if (tmp) c->release(tmp);
        return st;
      }
    }
  } else {
    if (e == hipSuccess) e = emb_import(c, dp, dv);
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, c->flag, 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  if (tmp) c->release(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "set_embedded: %s", hipGetErrorString(e));
  if (hbad & 4u) return fail(MPCD_EHIP, "set_embedded: the embedded-particle index is out of date");
  if (hbad & 1u) return fail(MPCD_EINVAL, "an embedded position lies outside [0, L)");
  return take_err(c);
}

mpcd_status mpcd_get_cells(mpcd_ctx c, int32_t* cell_of_tag, int32_t* counts, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (!c->have_bin) return fail(MPCD_ESTATE, "mpcd_get_cells: nothing has been binned");
  const size_t C = c->ncells;
  int32_t* dcell = cell_of_tag;
  int32_t* dcnt = counts;
  int32_t* tmp = nullptr;
  if (!on_device) {
    HIP_TRY(c->alloc((void**)&tmp, ((size_t)c->N + C) * 4 + 16));
    dcell = cell_of_tag ? tmp : nullptr;
    dcnt = counts ? tmp + c->N : nullptr;
  }
  hipError_t e = hipSuccess;
  if (dcnt && C) e = hipMemsetAsync(dcnt, 0, C * 4, c->stream);
  if (e == hipSuccess && c->N && (dcell || dcnt)) {
    if (ensure_shifts(c, c->last_bin_step, 1) != MPCD_OK) {
      if (tmp) c->release(tmp);
      return MPCD_EHIP;
    }
    const uint32_t nb = slab_blocks(c, c->S.cap);
    const ShiftEntry* sh = shift_at(c, c->last_bin_step);
    if (c->form == 0)
      k_cells<0><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->S, c->cnt[c->ci], sh, dcell, (uint32_t*)dcnt);
    else
      k_cells<1><<<nb, kGrid, 0, c->stream>>>(c->buf[c->cur], c->S, c->cnt[c->ci], sh, dcell, (uint32_t*)dcnt);
    e = hipGetLastError();
  }
  if (e == hipSuccess && tmp) {
    if (cell_of_tag && c->N) e = hipMemcpyAsync(cell_of_tag, dcell, (size_t)c->N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && counts && C) e = hipMemcpyAsync(counts, dcnt, C * 4, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) c->release(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "get_cells: %s", hipGetErrorString(e));
  return take_err(c);
}

static mpcd_status cell_diag(mpcd_ctx c, double* mass, double* mom, double* ek, double* axis,
                             double* xi, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (c->phase != Phase::Binned) return fail(MPCD_ESTATE, "cell diagnostics need the binned state");
  const size_t C = c->ncells;
  if (C == 0) return MPCD_OK;
  ST_TRY(ensure_shifts(c, c->step, 1));
  double* tmp = nullptr;
  HIP_TRY(c->alloc((void**)&tmp, C * 8 * 9));
  TileArgs a = tile_args(c);
  a.cnt_out = nullptr;
  a.cnt_clear = nullptr;
  a.step = (uint32_t)c->step;
  a.sh = shift_at(c, c->step);
  a.d_mass = tmp;
  a.d_mom = tmp + C;
  a.d_ek = tmp + 4 * C;
  a.d_axis = tmp + 5 * C;
  a.d_xi = tmp + 8 * C;
  hipError_t e = hipMemsetAsync(tmp, 0, C * 8 * 9, c->stream);
  if (e == hipSuccess) {
    if (c->form == 0) tile_dispatch<0>(c, a, MODE_DIAG, false);
    else tile_dispatch<1>(c, a, MODE_DIAG, false);
    e = hipGetLastError();
  }
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  struct {
    double* dst;
    double* src;
    size_t n;
  } cp[5] = {{mass, a.d_mass, C}, {mom, a.d_mom, 3 * C}, {ek, a.d_ek, C}, {axis, a.d_axis, 3 * C}, {xi, a.d_xi, C}};
  for (auto& q : cp)
    if (e == hipSuccess && q.dst) e = hipMemcpyAsync(q.dst, q.src, q.n * 8, kind, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->release(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "cell diagnostics: %s", hipGetErrorString(e));
  return take_err(c);
}

mpcd_status mpcd_get_cell_props(mpcd_ctx c, double* mass, double* momentum, double* ek,
                                int32_t on_device) {
  return cell_diag(c, mass, momentum, ek, nullptr, nullptr, on_device);
}

mpcd_status mpcd_get_cell_draws(mpcd_ctx c, double* axis, double* xi, int32_t on_device) {
  ST_TRY(check_ctx(c));
  if (c->p.collision == MPCD_AT) return fail(MPCD_EINVAL, "no per-cell draws under the AT rule");
  return cell_diag(c, nullptr, nullptr, nullptr, axis, xi, on_device);
}

mpcd_status mpcd_get_shift(mpcd_ctx c, uint64_t n, double s[3]) {
  ST_TRY(check_ctx(c));
  if (!s) return fail(MPCD_EINVAL, "s is NULL");
  shift_for(c, 0, n, s);
  return MPCD_OK;
}

mpcd_status mpcd_get_box(mpcd_ctx c, int32_t box, int64_t* first_tag, int64_t* n_particles,
                         int64_t* first_cell, int64_t* n_cells, double shift_of_step[3],
                         uint64_t step) {
  ST_TRY(check_ctx(c));
  if (box < 0 || (uint32_t)box >= c->nbox) return fail(MPCD_EINVAL, "box %d out of range", box);
  const Box& B = c->boxes[box];
  if (first_tag) *first_tag = B.tag0;
  if (n_particles) *n_particles = c->box_n[box];
  if (first_cell) *first_cell = B.cell0;
  if (n_cells) *n_cells = B.ncells;
  if (shift_of_step) shift_for(c, (uint32_t)box, step, shift_of_step);
  return MPCD_OK;
}

mpcd_status mpcd_get_velocity_field(mpcd_ctx c, double* u, double* mass, int32_t on_device) {
  ST_TRY(check_ctx(c));
  ST_TRY(materialize(c));  // the field pairs each particle's position with its velocity
  const size_t C = c->ncells;
  if (C == 0 || (!u && !mass)) return take_err(c);
  unsigned long long* acc = nullptr;
  HIP_TRY(c->alloc((void**)&acc, C * 64 + (on_device ? 0 : C * 32)));
  double* du = on_device ? u : (u ? (double*)(acc + 8 * C) : nullptr);
  double* dm = on_device ? mass : (mass ? (double*)(acc + 8 * C) + 3 * C : nullptr);
  hipError_t e = hipMemsetAsync(acc, 0, C * 64, c->stream);
  if (e == hipSuccess && c->N) {
    const uint32_t nb = slab_blocks(c, c->S.cap);
    const Particles P = c->buf[c->cur];
    const uint32_t* cn = c->cnt[c->ci];
    const bool em = c->n_emb > 0;
    if (c->form == 0) {
      if (em) k_field<0, true><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, acc, c->status);
      else k_field<0, false><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, acc, c->status);
    } else {
      if (em) k_field<1, true><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, acc, c->status);
      else k_field<1, false><<<nb, 256, 0, c->stream>>>(P, c->S, cn, c->emb_mass, acc, c->status);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_field_finish<<<blocks_for(C, 256), 256, 0, c->stream>>>(acc, C, du, dm);
    e = hipGetLastError();
  }
  if (e == hipSuccess && !on_device) {
    if (u) e = hipMemcpyAsync(u, du, C * 24, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && mass) e = hipMemcpyAsync(mass, dm, C * 8, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->release(acc);
  if (e != hipSuccess) return fail(MPCD_EHIP, "velocity field: %s", hipGetErrorString(e));
  return take_err(c);
}

mpcd_status mpcd_get_step(mpcd_ctx c, uint64_t* n) {
  ST_TRY(check_ctx(c));
  if (!n) return fail(MPCD_EINVAL, "n is NULL");
  *n = c->step;
  return MPCD_OK;
}

mpcd_status mpcd_set_step(mpcd_ctx c, uint64_t n) {
  ST_TRY(check_ctx(c));
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_set_step: only between steps");
  if (n >= 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  if (n != c->step) ST_TRY(drop_prepared(c));  // the prepared binning used step `step`'s shift
  c->step = n;
  return MPCD_OK;
}

mpcd_status mpcd_totals(mpcd_ctx c, double p[3], double* ke, double* kT) {
  ST_TRY(check_ctx(c));
  std::vector<long long> h;
  ST_TRY(read_totals(c, h));
  totals_of(c, h, 0, c->nbox, p, ke, kT);
  return take_err(c);
}

mpcd_status mpcd_box_totals(mpcd_ctx c, double* p, double* ke, double* kT) {
  ST_TRY(check_ctx(c));
  std::vector<long long> h;
  ST_TRY(read_totals(c, h));
  for (uint32_t b = 0; b < c->nbox; ++b)
    totals_of(c, h, b, b + 1, p ? p + 3 * b : nullptr, ke ? ke + b : nullptr, kT ? kT + b : nullptr);
  return take_err(c);
}

mpcd_status mpcd_sync(mpcd_ctx c) {
  ST_TRY(check_ctx(c));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return take_err(c);
}

mpcd_status mpcd_get_sizes(mpcd_ctx c, int64_t* n_total, int64_t* n_cells) {
  ST_TRY(check_ctx(c));
  if (n_total) *n_total = c->N;
  if (n_cells) *n_cells = (int64_t)c->ncells;
  return MPCD_OK;
}

mpcd_status mpcd_get_n_boxes(mpcd_ctx c, int32_t* n_boxes) {
  ST_TRY(check_ctx(c));
  if (n_boxes) *n_boxes = (int32_t)c->nbox;
  return MPCD_OK;
}

mpcd_status mpcd_footprint(const mpcd_params* params, int64_t n_particles, int64_t nsteps,
                           int32_t host_arrays, int64_t* peak_bytes, int64_t* held_bytes) {
  g_err.clear();
  ST_TRY(validate(params, n_particles, 0));
  if (nsteps < 0) return fail(MPCD_EINVAL, "nsteps < 0");
  Box B = make_box(*params);
  const double rho = B.ncells ? (double)n_particles / (double)B.ncells : 0.0;
  (void)choose_tiles(B, rho, tile_shape(*params), true,
                     params->collision == MPCD_AT && params->precision == MPCD_FP64);
  const uint64_t nt = B.ntiles, C = B.ncells, n = (uint64_t)n_particles;
  const bool fp64 = params->precision == MPCD_FP64;
  // every allocation is at least 256 bytes; allow that much again for the
  // pool's rounding
  auto sz = [](uint64_t bytes) { return std::max<uint64_t>(bytes, 256) + 256; };
  // the slab capacity mpcd_create picks when the fullest tile holds a whole
  // tile's mean occupancy plus five standard deviations (tiles cut by the
  // box's far faces hold fewer)
  const double full = rho * (double)B.td[0] * (double)B.td[1] * (double)B.td[2];
  const uint64_t cap = slab_cap((uint64_t)std::ceil(full + 5.0 * std::sqrt(full)),
                                (double)n / (double)nt);
  const uint64_t S = nt * cap;
  const uint64_t slabs = fp64 ? 2 * (3 * sz(S * 16) + sz(S * 4))   // wa wb wc, tag
                              : 2 * (2 * sz(S * 16));              // ra rb
  // counters (3), status, totals, embedded masses, box table, tile table, flag
  const uint64_t tables = 3 * sz(nt * 4) + sz(256) + sz(10 * 8) + sz(0) + sz(sizeof(Box)) +
                          sz(nt * 4) + sz(256);
  const uint64_t held = slabs + tables;
  const uint64_t shifts = sz(std::max<uint64_t>((uint64_t)nsteps + 1, 64) * sizeof(ShiftEntry));
  // temporaries, one at a time: the upload buffer of host arrays; the
  // readbacks' staging (state, cells, cell diagnostics, velocity field and
  // the join of a split state before it)
  const uint64_t upload = host_arrays ? sz(n * 48) : 0;
  const uint64_t h = host_arrays ? 1 : 0;
  const uint64_t readback = std::max({h * sz(n * 48), h * sz((n + C) * 4 + 16), sz(C * 72),
                                      sz(C * (64 + 32 * h)), sz(n * 3 * (fp64 ? 8 : 4))});
  const uint64_t peak = held + std::max(upload, shifts + readback);
  if (peak_bytes) *peak_bytes = (int64_t)peak;
  if (held_bytes) *held_bytes = (int64_t)(held + shifts);
  return MPCD_OK;
}

mpcd_status mpcd_get_layout(mpcd_ctx c, int32_t tile[3], int64_t* n_tiles, int64_t* capacity,
                            int64_t* regrows) {
  ST_TRY(check_ctx(c));
  if (tile)
    for (int d = 0; d < 3; ++d) tile[d] = c->boxes[0].td[d];
  if (n_tiles) *n_tiles = c->S.ntiles;
  if (capacity) *capacity = c->S.cap;
  if (regrows) *regrows = c->regrows;
  return MPCD_OK;
}

mpcd_status mpcd_debug_fail_allocs(int64_t after, int64_t count) {
  if (after < 0 || count <= 0) {
    g_fail_after.store(-1);
    g_fail_count.store(0);
    return MPCD_OK;
  }
  g_fail_count.store(count);
  g_fail_after.store(after);
  return MPCD_OK;
}

mpcd_status mpcd_handover_stats(mpcd_ctx c, int64_t* kept, int64_t* given_up) {
  ST_TRY(check_ctx(c));
  if (kept) *kept = (int64_t)c->handovers[0];
  if (given_up) *given_up = (int64_t)c->handovers[1];
  return MPCD_OK;
}

mpcd_status mpcd_set_graph(mpcd_ctx c, int32_t on) {
  ST_TRY(check_ctx(c));
  if (on != 0 && on != 1) return fail(MPCD_EINVAL, "on must be 0 or 1");
  if (on && (c->stream == nullptr || c->stream == hipStreamPerThread))
    return fail(MPCD_EINVAL, "graph launches need a stream other than the null or per-thread stream");
  c->graph = on != 0;
  return MPCD_OK;
}

mpcd_status mpcd_graph_stats(mpcd_ctx c, int64_t* instantiations, int64_t* updates) {
  ST_TRY(check_ctx(c));
  if (instantiations) *instantiations = (int64_t)c->graph_inst;
  if (updates) *updates = (int64_t)c->graph_upd;
  return MPCD_OK;
}

mpcd_status mpcd_profile_enable(mpcd_ctx c, int32_t on) {
  ST_TRY(check_ctx(c));
  if (on < 0) return fail(MPCD_EINVAL, "profile period < 0");
  c->prof_every = on;
  for (uint64_t& n : c->prof_seen) n = 0;
  return MPCD_OK;
}

mpcd_status mpcd_profile_read(mpcd_ctx c, int32_t which, double* total_ms, int64_t* launches) {
  ST_TRY(check_ctx(c));
  if (which < 0 || which > 1) return fail(MPCD_EINVAL, "which must be 0 or 1");
  HIP_TRY(hipStreamSynchronize(c->stream));
  double ms = 0.0;
  auto& v = c->ev_used[which];
  for (auto& pr : v) {
    float t = 0.0f;
    HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
    ms += t;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = (int64_t)v.size();
  v.clear();
  return MPCD_OK;
}

mpcd_status mpcd_philox4x32_10(const uint32_t* ctr, int64_t n, uint64_t key, uint32_t* out) {
  g_err.clear();
  if (n < 0 || n > (1ll << 30)) return fail(MPCD_EINVAL, "n out of range");
  if (n == 0) return MPCD_OK;
  if (!ctr || !out) return fail(MPCD_EINVAL, "NULL pointer");
  U4 *dc = nullptr, *dout = nullptr;
  HIP_TRY(hipMalloc(&dc, (size_t)n * 16));
  hipError_t e = hipMalloc(&dout, (size_t)n * 16);
  if (e == hipSuccess) e = hipMemcpy(dc, ctr, (size_t)n * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    k_philox<<<blocks_for(n, 256), 256>>>(dc, (uint32_t)n, (uint32_t)key, (uint32_t)(key >> 32), dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, dout, (size_t)n * 16, hipMemcpyDeviceToHost);
  (void)hipFree(dc);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return fail(MPCD_EHIP, "philox: %s", hipGetErrorString(e));
  return MPCD_OK;
}

}  // extern "C"

static mpcd_status copy_impl(const void* src, void* dst, int64_t bytes, void* hip_stream,
                             bool unrolled) {
  g_err.clear();
  if (bytes < 0 || (!src && bytes) || (!dst && bytes)) return fail(MPCD_EINVAL, "bad copy arguments");
  if (bytes == 0) return MPCD_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  const bool aligned = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
  const size_t n16 = aligned ? (size_t)bytes / 16 : 0;
  if (n16) {
    if (unrolled) {
      const uint32_t nb = (uint32_t)std::min<size_t>((n16 + 1023) / 1024, 256u * 256u);
      k_copy16x4<<<nb, 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
    } else {
      const uint32_t nb = (uint32_t)std::min<size_t>((n16 + 255) / 256, 256u * 256u);
      k_copy16<<<nb, 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
    }
  }
  const size_t tail = (size_t)bytes - n16 * 16;
  if (tail)
    k_copy1<<<blocks_for(tail, 256), 256, 0, s>>>((const unsigned char*)src + n16 * 16,
                                                  (unsigned char*)dst + n16 * 16, tail);
  HIP_TRY(hipGetLastError());
  return MPCD_OK;
}

extern "C" {

mpcd_status mpcd_md_verlet_chains(double* pos, double* vel, const double* mass, int64_t n_chains,
                                  int32_t chain_len, const double box[3], double k_bond,
                                  double bond_length, double dt, int32_t nsteps, void* hip_stream) {
  g_err.clear();
  if (n_chains < 0 || nsteps < 0) return fail(MPCD_EINVAL, "n_chains and nsteps must be >= 0");
  if (chain_len < 1 || chain_len > 1024) return fail(MPCD_EINVAL, "chain_len must be 1..1024");
  if (n_chains > 0x7FFFFFFF) return fail(MPCD_EINVAL, "too many chains");
  if (!box || !(box[0] > 0.0) || !(box[1] > 0.0) || !(box[2] > 0.0))
    return fail(MPCD_EINVAL, "box lengths must be > 0");
  if (!std::isfinite(k_bond) || !std::isfinite(bond_length) || !(dt >= 0.0) || !std::isfinite(dt))
    return fail(MPCD_EINVAL, "k_bond, bond_length must be finite and dt >= 0");
  if (n_chains == 0 || nsteps == 0) return MPCD_OK;
  if (!pos || !vel || !mass) return fail(MPCD_EINVAL, "pos/vel/mass NULL");
  const uint32_t threads = ((uint32_t)chain_len + 63u) / 64u * 64u;
  const size_t lds = (size_t)chain_len * 3 * sizeof(double);
  hipStream_t st = (hipStream_t)hip_stream;
  k_md_chains<<<(uint32_t)n_chains, threads, lds, st>>>(pos, vel, mass, (uint32_t)chain_len, box[0], box[1],
                                                        box[2], k_bond, bond_length, dt, nsteps);
  HIP_TRY(hipGetLastError());
  return MPCD_OK;
}

mpcd_status mpcd_copy_kernel(const void* src, void* dst, int64_t bytes, void* hip_stream) {
  return copy_impl(src, dst, bytes, hip_stream, false);
}

mpcd_status mpcd_copy_kernel_unrolled(const void* src, void* dst, int64_t bytes, void* hip_stream) {
  return copy_impl(src, dst, bytes, hip_stream, true);
}

}  // extern "C"
