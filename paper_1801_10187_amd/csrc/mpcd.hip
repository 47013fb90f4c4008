// libmpcd: host side of the C ABI declared in include/mpcd.h.
//
// The context owns every device buffer (hipMalloc at create, hipFree at
// destroy) and enqueues all work on one HIP stream. A step is launched as
//   stream+bin (first step only) | scan -> list -> collide(+stream+bin next)
// so that after the first step every step costs one pass over the particles
// plus the small per-cell scan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mpcd.h"
#include "mpcd_kernels.hpp"

using namespace mpcd;

namespace {

thread_local std::string g_err;

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
      return fail(MPCD_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

enum class Phase { Idle, Streamed, Binned };

constexpr uint32_t kGrid = 256;  // threads per block of the elementwise kernels

inline uint32_t blocks_for(uint64_t n, uint32_t per) {
  return (uint32_t)((n + per - 1) / per);
}

}  // namespace

struct mpcd_ctx_s {
  mpcd_params p{};
  int form = 0;
  uint32_t n_solv = 0, n_emb = 0, N = 0;
  Box box{};
  int cpb = 128;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;

  // device memory
  std::vector<void*> allocs;
  Particles buf[2]{};
  int cur = 0;
  uint2* cr = nullptr;
  uint32_t* perm = nullptr;
  uint32_t* count = nullptr;
  uint32_t* off = nullptr;
  uint32_t* partial = nullptr;
  uint32_t n_partial = 0;
  double* emb_mass = nullptr;
  uint32_t* err = nullptr;
  long long* tot = nullptr;

  uint64_t step = 0;
  Phase phase = Phase::Idle;
  bool have_bin = false;       // a binning has happened
  bool sorted_by_bin = false;  // current buffer is in the cell order of the last bin

  // profiling: pairs of events per instrumented launch
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[3];

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    allocs.push_back(p);
    return p;
  }
};

namespace {

mpcd_status check_ctx(mpcd_ctx c) {
  if (!c) return fail(MPCD_EINVAL, "null context");
  return MPCD_OK;
}

mpcd_status take_err(mpcd_ctx c) {
  uint32_t e = 0;
  HIP_TRY(hipMemcpyAsync(&e, c->err, sizeof e, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (e) {
    HIP_TRY(hipMemsetAsync(c->err, 0, sizeof e, c->stream));
    return fail(MPCD_ERANGE, "kernel range check failed (flags 0x%x: %s%s%s%s)", e,
                (e & ERR_STREAM_RANGE) ? "displacement >= box length; " : "",
                (e & ERR_FIXED_RANGE) ? "value outside fixed-point range; " : "",
                (e & ERR_GAMMA_CAP) ? "Gamma sampler attempt cap; " : "",
                (e & ERR_LIST) ? "cell list inconsistent; " : "");
  }
  return MPCD_OK;
}

void shift_for(const mpcd_ctx c, uint64_t n, double s[3], float s32[3]) {
  if (c->p.grid_shift) {
    grid_shift(c->box.k0, c->box.k1, (uint32_t)n, c->p.a, s);
  } else {
    s[0] = s[1] = s[2] = 0.0;
  }
  for (int d = 0; d < 3; ++d) s32[d] = (float)s[d];
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
    if (!c->prof) return;
    e0 = pool_event(c);
    e1 = pool_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, c->stream);
  }
  ~ProfScope() {
    if (!c->prof || !e0 || !e1) return;
    (void)hipEventRecord(e1, c->stream);
    c->ev_used[which].emplace_back(e0, e1);
  }
};

// --- launch wrappers
mpcd_status launch_stream(mpcd_ctx c) {
  if (c->N == 0) return MPCD_OK;
  ProfScope ps(c, 1);
  if (c->form == 0)
    k_stream<0><<<blocks_for(c->N, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur], c->box, c->N, c->err);
  else
    k_stream<1><<<blocks_for(c->N, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur], c->box, c->N, c->err);
  HIP_TRY(hipGetLastError());
  return MPCD_OK;
}

mpcd_status launch_bin(mpcd_ctx c, bool with_stream) {
  if (c->N == 0) return MPCD_OK;
  double s[3];
  float s32[3];
  shift_for(c, c->step, s, s32);
  ProfScope ps(c, 1);
  const uint32_t nb = blocks_for(c->N, kGrid);
  Particles& P = c->buf[c->cur];
#define BIN_LAUNCH(F, S)                                                                   \
  k_bin<F, S><<<nb, kGrid, 0, c->stream>>>(P, c->box, c->N, s[0], s[1], s[2], s32[0], s32[1], \
                                           s32[2], c->count, c->cr, c->err)
  if (c->form == 0) {
    if (with_stream) BIN_LAUNCH(0, true); else BIN_LAUNCH(0, false);
  } else {
    if (with_stream) BIN_LAUNCH(1, true); else BIN_LAUNCH(1, false);
  }
#undef BIN_LAUNCH
  HIP_TRY(hipGetLastError());
  return MPCD_OK;
}

// counts -> offsets (count cleared), then the cell-ordered list
mpcd_status launch_scan_list(mpcd_ctx c) {
  ProfScope ps(c, 2);
  const uint32_t C = c->box.ncells;
  const uint32_t nb = c->n_partial;
  k_scan_partial<<<nb, SCAN_T, 0, c->stream>>>(c->count, C, c->partial);
  k_scan_top<<<1, 1024, 0, c->stream>>>(c->partial, nb);
  k_scan_final<<<nb, SCAN_T, 0, c->stream>>>(c->count, C, c->partial, c->off, c->N);
  if (c->N) k_perm<<<blocks_for(c->N, kGrid), kGrid, 0, c->stream>>>(c->cr, c->off, c->perm, c->N, c->err);
  HIP_TRY(hipGetLastError());
  return MPCD_OK;
}

template <int F, int CPB, bool SN, bool TH, bool EM>
void collide_inst(mpcd_ctx c, const CollideArgs& a) {
  const uint32_t nb = blocks_for(c->box.ncells, CPB);
  k_collide<F, CPB, SN, TH, EM><<<nb, COLLIDE_T, 0, c->stream>>>(a);
}

template <int F, int CPB>
void collide_dispatch3(mpcd_ctx c, const CollideArgs& a, bool sn, bool th, bool em) {
  if (sn) {
    if (th) { if (em) collide_inst<F, CPB, true, true, true>(c, a); else collide_inst<F, CPB, true, true, false>(c, a); }
    else    { if (em) collide_inst<F, CPB, true, false, true>(c, a); else collide_inst<F, CPB, true, false, false>(c, a); }
  } else {
    if (th) { if (em) collide_inst<F, CPB, false, true, true>(c, a); else collide_inst<F, CPB, false, true, false>(c, a); }
    else    { if (em) collide_inst<F, CPB, false, false, true>(c, a); else collide_inst<F, CPB, false, false, false>(c, a); }
  }
}

template <int F>
void collide_dispatch(mpcd_ctx c, const CollideArgs& a, bool sn, bool th, bool em) {
  switch (c->cpb) {
    case 256: collide_dispatch3<F, 256>(c, a, sn, th, em); break;
    case 64: collide_dispatch3<F, 64>(c, a, sn, th, em); break;
    default: collide_dispatch3<F, 128>(c, a, sn, th, em); break;
  }
}

// collide with counter c->step; with stream_next, stream and bin for
// c->step + 1 as well. Swaps the particle buffers.
mpcd_status launch_collide(mpcd_ctx c, bool stream_next) {
  CollideArgs a{};
  a.cur = c->buf[c->cur];
  a.nxt = c->buf[1 - c->cur];
  a.B = c->box;
  a.off = c->off;
  a.perm = c->perm;
  a.emb_mass = c->emb_mass;
  a.step = (uint32_t)c->step;
  a.step_next = (uint32_t)(c->step + 1);
  shift_for(c, c->step + 1, a.sn, a.sn32);
  a.count = c->count;
  a.cr_next = c->cr;
  a.err = c->err;
  if (c->box.ncells > 0) {
    ProfScope ps(c, 0);
    const bool th = c->p.thermostat != 0, em = c->n_emb > 0;
    if (c->form == 0) collide_dispatch<0>(c, a, stream_next, th, em);
    else collide_dispatch<1>(c, a, stream_next, th, em);
    HIP_TRY(hipGetLastError());
  }
  c->cur = 1 - c->cur;
  return MPCD_OK;
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
  if (p->flags != 0) return fail(MPCD_EINVAL, "flags must be 0");
  if (p->precision == MPCD_FP32)
    for (int d = 0; d < 3; ++d)
      if (p->n_cells[d] > 1024) return fail(MPCD_EINVAL, "FP32 form supports at most 1024 cells per axis");
  if (ns < 0 || ne < 0) return fail(MPCD_EINVAL, "negative particle count");
  if (ns + ne >= (int64_t)1 << 31) return fail(MPCD_EINVAL, "at most 2^31 - 1 particles");
  return MPCD_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* mpcd_last_error(void) { return g_err.c_str(); }

mpcd_status mpcd_create(const mpcd_params* params, int64_t n_solvent, const double* pos,
                        const double* vel, int64_t n_embedded, const double* emb_pos,
                        const double* emb_vel, const double* emb_mass,
                        int32_t pointers_on_device, void* hip_stream, mpcd_ctx* out) {
  g_err.clear();
  if (!out) return fail(MPCD_EINVAL, "out is NULL");
  *out = nullptr;
  mpcd_status st = validate(params, n_solvent, n_embedded);
  if (st != MPCD_OK) return st;
  if (n_solvent > 0 && (!pos || !vel)) return fail(MPCD_EINVAL, "pos/vel NULL");
  if (n_embedded > 0 && (!emb_pos || !emb_vel || !emb_mass))
    return fail(MPCD_EINVAL, "embedded arrays NULL");
  std::vector<double> hmass;
  if (n_embedded > 0 && !pointers_on_device) {
    for (int64_t i = 0; i < n_embedded; ++i)
      if (!(emb_mass[i] > 0.0) || !std::isfinite(emb_mass[i]))
        return fail(MPCD_EINVAL, "embedded mass %lld is not > 0", (long long)i);
  }

  mpcd_ctx c = new (std::nothrow) mpcd_ctx_s();
  if (!c) return fail(MPCD_ENOMEM, "host allocation failed");
  auto cleanup = [&](mpcd_status s) {
    mpcd_destroy(c);
    return s;
  };
  c->p = *params;
  c->form = params->precision;
  c->n_solv = (uint32_t)n_solvent;
  c->n_emb = (uint32_t)n_embedded;
  c->N = (uint32_t)(n_solvent + n_embedded);
  Box& B = c->box;
  for (int d = 0; d < 3; ++d) {
    B.n[d] = params->n_cells[d];
    B.L[d] = (double)params->n_cells[d] * params->a;
  }
  B.a = params->a;
  B.inv_a = 1.0 / params->a;
  B.dt = params->dt;
  B.a32 = (float)params->a;
  B.inv_a32 = (float)B.inv_a;
  B.dt32 = (float)params->dt;
  B.ncells = (uint32_t)((uint64_t)params->n_cells[0] * params->n_cells[1] * params->n_cells[2]);
  B.ca = std::cos(params->alpha);
  B.sa = std::sin(params->alpha);
  B.omc = 1.0 - B.ca;
  B.kT = params->kT;
  B.mass = params->solvent_mass;
  B.k0 = (uint32_t)(params->seed & 0xFFFFFFFFull);
  B.k1 = (uint32_t)(params->seed >> 32);
  B.n_solvent = c->n_solv;
  const double rho = B.ncells ? (double)c->N / (double)B.ncells : 0.0;
  c->cpb = rho * 256.0 <= 1400.0 ? 256 : (rho * 128.0 <= 1400.0 ? 128 : 64);

  if (hipGetDevice(&c->device) != hipSuccess) return cleanup(fail(MPCD_EHIP, "no HIP device"));
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return cleanup(fail(MPCD_EHIP, "hipStreamCreate failed"));
    c->own_stream = true;
  }

  const size_t N = c->N;
  const size_t C = B.ncells;
  for (int b = 0; b < 2; ++b) {
    Particles& P = c->buf[b];
    if (c->form == 0) {
      for (int d = 0; d < 3; ++d) {
        P.x[d] = (double*)c->dalloc(N * 8);
        P.v[d] = (double*)c->dalloc(N * 8);
        if (!P.x[d] || !P.v[d]) return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
      }
    } else {
      P.h = (uint32_t*)c->dalloc(N * 4);
      if (!P.h) return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
      for (int d = 0; d < 3; ++d) {
        P.o[d] = (float*)c->dalloc(N * 4);
        P.vf[d] = (float*)c->dalloc(N * 4);
        if (!P.o[d] || !P.vf[d]) return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
      }
    }
    P.tag = (uint32_t*)c->dalloc(N * 4);
    if (!P.tag) return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
  }
  c->n_partial = blocks_for(C, SCAN_CHUNK);
  c->cr = (uint2*)c->dalloc(N * 8);
  c->perm = (uint32_t*)c->dalloc(N * 4);
  c->count = (uint32_t*)c->dalloc(C * 4 + 64);
  c->off = (uint32_t*)c->dalloc(C * 4 + 64);
  c->partial = (uint32_t*)c->dalloc((size_t)c->n_partial * 4);
  c->err = (uint32_t*)c->dalloc(256);
  c->tot = (long long*)c->dalloc(10 * 8);
  c->emb_mass = (double*)c->dalloc((size_t)c->n_emb * 8);
  if (!c->cr || !c->perm || !c->count || !c->off || !c->partial || !c->err || !c->tot ||
      !c->emb_mass)
    return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
  if (hipMemsetAsync(c->count, 0, C * 4 + 64, c->stream) != hipSuccess ||
      hipMemsetAsync(c->err, 0, 256, c->stream) != hipSuccess)
    return cleanup(fail(MPCD_EHIP, "hipMemset failed"));

  // import: host arrays are staged through a temporary device buffer
  uint32_t* bad = (uint32_t*)c->dalloc(256);
  if (!bad || hipMemsetAsync(bad, 0, 256, c->stream) != hipSuccess)
    return cleanup(fail(MPCD_ENOMEM, "device allocation failed"));
  auto import = [&](const double* hp, const double* hv, uint32_t n, uint32_t tag0) -> mpcd_status {
    if (n == 0) return MPCD_OK;
    const double* dp = hp;
    const double* dv = hv;
    double* tmp = nullptr;
    if (!pointers_on_device) {
      if (hipMalloc(&tmp, (size_t)n * 48) != hipSuccess)
        return fail(MPCD_ENOMEM, "device allocation of the upload buffer failed");
      if (hipMemcpyAsync(tmp, hp, (size_t)n * 24, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
          hipMemcpyAsync(tmp + 3 * (size_t)n, hv, (size_t)n * 24, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        (void)hipFree(tmp);
        return fail(MPCD_EHIP, "upload failed");
      }
      dp = tmp;
      dv = tmp + 3 * (size_t)n;
    }
    if (c->form == 0)
      k_import<0><<<blocks_for(n, kGrid), kGrid, 0, c->stream>>>(c->buf[0], B, dp, dv, n, tag0, bad);
    else
      k_import<1><<<blocks_for(n, kGrid), kGrid, 0, c->stream>>>(c->buf[0], B, dp, dv, n, tag0, bad);
    hipError_t e = hipGetLastError();
    if (tmp) {
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(tmp);
    }
    if (e != hipSuccess) return fail(MPCD_EHIP, "import kernel: %s", hipGetErrorString(e));
    return MPCD_OK;
  };
  if ((st = import(pos, vel, c->n_solv, 0)) != MPCD_OK) return cleanup(st);
  if ((st = import(emb_pos, emb_vel, c->n_emb, c->n_solv)) != MPCD_OK) return cleanup(st);
  if (c->n_emb) {
    if (hipMemcpyAsync(c->emb_mass, emb_mass, (size_t)c->n_emb * 8,
                       pointers_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       c->stream) != hipSuccess)
      return cleanup(fail(MPCD_EHIP, "upload of embedded masses failed"));
  }
  uint32_t hbad = 0;
  if (hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return cleanup(fail(MPCD_EHIP, "create: synchronisation failed"));
  if (hbad) return cleanup(fail(MPCD_EINVAL, "a position lies outside [0, L)"));
  c->cur = 0;
  c->step = 0;
  c->phase = Phase::Idle;
  *out = c;
  return MPCD_OK;
}

void mpcd_destroy(mpcd_ctx c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void* p : c->allocs) (void)hipFree(p);
  for (auto& v : c->ev_used)
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

mpcd_status mpcd_stream(mpcd_ctx c) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_stream: expected the state after create or collide");
  if ((st = launch_stream(c)) != MPCD_OK) return st;
  c->phase = Phase::Streamed;
  return MPCD_OK;
}

mpcd_status mpcd_bin(mpcd_ctx c) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (c->phase != Phase::Streamed) return fail(MPCD_ESTATE, "mpcd_bin: expected a preceding mpcd_stream");
  if (c->step >= 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  if ((st = launch_bin(c, false)) != MPCD_OK) return st;
  if ((st = launch_scan_list(c)) != MPCD_OK) return st;
  c->phase = Phase::Binned;
  c->have_bin = true;
  c->sorted_by_bin = false;
  return MPCD_OK;
}

mpcd_status mpcd_collide(mpcd_ctx c) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (c->phase != Phase::Binned) return fail(MPCD_ESTATE, "mpcd_collide: expected a preceding mpcd_bin");
  if ((st = launch_collide(c, false)) != MPCD_OK) return st;
  c->step += 1;
  c->phase = Phase::Idle;
  c->sorted_by_bin = true;
  return MPCD_OK;
}

mpcd_status mpcd_step(mpcd_ctx c, int64_t nsteps) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (nsteps < 0) return fail(MPCD_EINVAL, "nsteps < 0");
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_step: expected the state after create or collide");
  if (nsteps == 0) return MPCD_OK;
  if (c->step + (uint64_t)nsteps > 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  if ((st = launch_bin(c, true)) != MPCD_OK) return st;
  for (int64_t k = 0; k < nsteps; ++k) {
    if ((st = launch_scan_list(c)) != MPCD_OK) return st;
    if ((st = launch_collide(c, k + 1 < nsteps)) != MPCD_OK) return st;
    c->step += 1;
  }
  c->have_bin = true;
  c->sorted_by_bin = true;
  c->phase = Phase::Idle;
  return MPCD_OK;
}

mpcd_status mpcd_get_state(mpcd_ctx c, double* pos, double* vel, int32_t on_device) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (!pos || !vel) return fail(MPCD_EINVAL, "pos/vel NULL");
  if (c->N == 0) return take_err(c);
  double* dp = pos;
  double* dv = vel;
  double* tmp = nullptr;
  if (!on_device) {
    HIP_TRY(hipMalloc(&tmp, (size_t)c->N * 48));
    dp = tmp;
    dv = tmp + 3 * (size_t)c->N;
  }
  if (c->form == 0)
    k_export<0><<<blocks_for(c->N, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur], c->box, c->N, dp, dv);
  else
    k_export<1><<<blocks_for(c->N, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur], c->box, c->N, dp, dv);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && tmp) {
    e = hipMemcpyAsync(pos, dp, (size_t)c->N * 24, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(vel, dv, (size_t)c->N * 24, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "get_state: %s", hipGetErrorString(e));
  return take_err(c);
}

mpcd_status mpcd_get_cells(mpcd_ctx c, int32_t* cell_of_tag, int32_t* counts, int32_t on_device) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (!c->have_bin) return fail(MPCD_ESTATE, "mpcd_get_cells: nothing has been binned");
  const size_t C = c->box.ncells;
  int32_t* dcell = cell_of_tag;
  int32_t* dcnt = counts;
  int32_t* tmp = nullptr;
  if (!on_device) {
    HIP_TRY(hipMalloc(&tmp, ((size_t)c->N + C) * 4 + 16));
    dcell = cell_of_tag ? tmp : nullptr;
    dcnt = counts ? tmp + c->N : nullptr;
  }
  if (c->sorted_by_bin) {
    if (C) k_cells_from_order<<<blocks_for(C, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur].tag, c->off, (uint32_t)C, dcell, dcnt);
  } else {
    if (dcell && c->N)
      k_cells_from_cr<<<blocks_for(c->N, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur].tag, c->cr, c->N, dcell);
    if (dcnt && C)
      k_cells_from_order<<<blocks_for(C, kGrid), kGrid, 0, c->stream>>>(c->buf[c->cur].tag, c->off, (uint32_t)C, nullptr, dcnt);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && tmp) {
    if (cell_of_tag && c->N) e = hipMemcpyAsync(cell_of_tag, dcell, (size_t)c->N * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && counts && C) e = hipMemcpyAsync(counts, dcnt, C * 4, hipMemcpyDeviceToHost, c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (tmp) (void)hipFree(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "get_cells: %s", hipGetErrorString(e));
  return take_err(c);
}

static mpcd_status cell_diag(mpcd_ctx c, double* mass, double* mom, double* ek, double* axis,
                             double* xi, int32_t on_device) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (c->phase != Phase::Binned) return fail(MPCD_ESTATE, "cell diagnostics need the binned state");
  const size_t C = c->box.ncells;
  if (C == 0) return MPCD_OK;
  double* tmp = nullptr;
  HIP_TRY(hipMalloc(&tmp, C * 8 * 9));
  double *dm = tmp, *dmom = tmp + C, *dek = tmp + 4 * C, *dax = tmp + 5 * C, *dxi = tmp + 8 * C;
  const bool th = c->p.thermostat != 0, em = c->n_emb > 0;
  const uint32_t nb = blocks_for(C, kGrid);
  const Particles P = c->buf[c->cur];
#define DIAG(F, T, E)                                                                     \
  k_cell_diag<F, T, E><<<nb, kGrid, 0, c->stream>>>(P, c->box, c->off, c->perm, c->emb_mass, \
                                                    (uint32_t)c->step, dm, dek, dax, dxi, c->err)
#define MOM(F, E) \
  k_cell_momentum<F, E><<<nb, kGrid, 0, c->stream>>>(P, c->box, c->off, c->perm, c->emb_mass, dmom, c->err)
  if (c->form == 0) {
    if (th) { if (em) DIAG(0, true, true); else DIAG(0, true, false); }
    else    { if (em) DIAG(0, false, true); else DIAG(0, false, false); }
    if (em) MOM(0, true); else MOM(0, false);
  } else {
    if (th) { if (em) DIAG(1, true, true); else DIAG(1, true, false); }
    else    { if (em) DIAG(1, false, true); else DIAG(1, false, false); }
    if (em) MOM(1, true); else MOM(1, false);
  }
#undef DIAG
#undef MOM
  hipError_t e = hipGetLastError();
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  struct { double* dst; double* src; size_t n; } cp[5] = {
      {mass, dm, C}, {mom, dmom, 3 * C}, {ek, dek, C}, {axis, dax, 3 * C}, {xi, dxi, C}};
  for (auto& q : cp)
    if (e == hipSuccess && q.dst) e = hipMemcpyAsync(q.dst, q.src, q.n * 8, kind, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail(MPCD_EHIP, "cell diagnostics: %s", hipGetErrorString(e));
  return take_err(c);
}

mpcd_status mpcd_get_cell_props(mpcd_ctx c, double* mass, double* momentum, double* ek,
                                int32_t on_device) {
  return cell_diag(c, mass, momentum, ek, nullptr, nullptr, on_device);
}

mpcd_status mpcd_get_cell_draws(mpcd_ctx c, double* axis, double* xi, int32_t on_device) {
  return cell_diag(c, nullptr, nullptr, nullptr, axis, xi, on_device);
}

mpcd_status mpcd_get_shift(mpcd_ctx c, uint64_t n, double s[3]) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (!s) return fail(MPCD_EINVAL, "s is NULL");
  float s32[3];
  shift_for(c, n, s, s32);
  return MPCD_OK;
}

mpcd_status mpcd_get_step(mpcd_ctx c, uint64_t* n) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (!n) return fail(MPCD_EINVAL, "n is NULL");
  *n = c->step;
  return MPCD_OK;
}

mpcd_status mpcd_set_step(mpcd_ctx c, uint64_t n) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (c->phase != Phase::Idle) return fail(MPCD_ESTATE, "mpcd_set_step: only between steps");
  if (n >= 0xFFFFFFFFull) return fail(MPCD_ERANGE, "step counter beyond 2^32 - 1");
  c->step = n;
  return MPCD_OK;
}

mpcd_status mpcd_totals(mpcd_ctx c, double p[3], double* ke, double* kT) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  long long h[10] = {0};
  if (c->N) {
    HIP_TRY(hipMemsetAsync(c->tot, 0, 80, c->stream));
    const uint32_t nb = std::min<uint32_t>(blocks_for(c->N, kGrid), 2048u);
    const bool em = c->n_emb > 0;
    const Particles P = c->buf[c->cur];
    if (c->form == 0) {
      if (em) k_totals<0, true><<<nb, 256, 0, c->stream>>>(P, c->box, c->N, c->emb_mass, c->tot, c->err);
      else k_totals<0, false><<<nb, 256, 0, c->stream>>>(P, c->box, c->N, c->emb_mass, c->tot, c->err);
    } else {
      if (em) k_totals<1, true><<<nb, 256, 0, c->stream>>>(P, c->box, c->N, c->emb_mass, c->tot, c->err);
      else k_totals<1, false><<<nb, 256, 0, c->stream>>>(P, c->box, c->N, c->emb_mass, c->tot, c->err);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h, c->tot, 80, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  auto val = [&](int q) { return (double)h[2 * q] * 0x1p-20 + (double)h[2 * q + 1] * 0x1p-72; };
  const double P0 = val(0), P1 = val(1), P2 = val(2), K = 0.5 * val(3), M = val(4);
  if (p) {
    p[0] = P0;
    p[1] = P1;
    p[2] = P2;
  }
  if (ke) *ke = K;
  if (kT) *kT = (c->N > 1 && M > 0) ? 2.0 * (K - 0.5 * (P0 * P0 + P1 * P1 + P2 * P2) / M) / (3.0 * (c->N - 1)) : 0.0;
  return take_err(c);
}

mpcd_status mpcd_sync(mpcd_ctx c) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return take_err(c);
}

mpcd_status mpcd_get_sizes(mpcd_ctx c, int64_t* n_total, int64_t* n_cells) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (n_total) *n_total = c->N;
  if (n_cells) *n_cells = c->box.ncells;
  return MPCD_OK;
}

mpcd_status mpcd_profile_enable(mpcd_ctx c, int32_t on) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  c->prof = on != 0;
  return MPCD_OK;
}

mpcd_status mpcd_profile_read(mpcd_ctx c, int32_t which, double* total_ms, int64_t* launches) {
  mpcd_status st = check_ctx(c);
  if (st) return st;
  if (which < 0 || which > 2) return fail(MPCD_EINVAL, "which must be 0, 1 or 2");
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

mpcd_status mpcd_copy_kernel(const void* src, void* dst, int64_t bytes, void* hip_stream) {
  g_err.clear();
  if (bytes < 0 || (!src && bytes) || (!dst && bytes)) return fail(MPCD_EINVAL, "bad copy arguments");
  if (bytes == 0) return MPCD_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  const bool aligned = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
  const size_t n16 = aligned ? (size_t)bytes / 16 : 0;
  if (n16) {
    const uint32_t nb = (uint32_t)std::min<size_t>((n16 + 255) / 256, 256u * 256u);
    k_copy16<<<nb, 256, 0, s>>>((const uint4*)src, (uint4*)dst, n16);
  }
  const size_t tail = (size_t)bytes - n16 * 16;
  if (tail)
    k_copy1<<<blocks_for(tail, 256), 256, 0, s>>>((const unsigned char*)src + n16 * 16,
                                                  (unsigned char*)dst + n16 * 16, tail);
  HIP_TRY(hipGetLastError());
  return MPCD_OK;
}

}  // extern "C"
