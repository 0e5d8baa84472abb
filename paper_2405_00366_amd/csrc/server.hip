// Serving form: continuous batching of L0RBCS solves (Algorithm 1) over one
// caller-provided device arena.
//
// Requests are queued on submit.  Each tick admits queued requests in
// arrival order while a slot is free, the request's footprint fits in the
// arena (first fit) and, when the caller set one, the couplings bytes that
// one Euler step of the resident set streams stay within the step budget;
// then advances every resident request by one
// alternation of Algorithm 1 (couplings, one CIM run, replica choice, Jacobi
// CDP) with the batched kernels: requests of different N, M and sparsity
// share every launch, each with its own alternation index, eta and random
// stream.  Requests that have done all their alternations are reported
// (eq. 3 objective, optional FP64 refit), their outputs copied to the
// caller's buffers, and their memory and slot returned before the next
// tick.  A request's arithmetic depends only on its own data, so its result
// is the same alone and in any mix.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include "batch.h"
#include "serve_sched.h"

using namespace l0;

namespace {

int round_up32(int x) { return (x + 31) / 32 * 32; }

// Byte offsets of one request's arrays inside its arena block.
struct ReqLayout {
  size_t G, Gc, J, b, z, rs, R, sig, c, c2, e, xb, xb2, sig_all, hpart, jw, A, y, total;
};

ReqLayout req_layout(int m, int n, int P, size_t jsz) {
  const size_t ld = size_t(round_up32(n));
  ReqLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.G = take(size_t(n) * ld * 4);
  L.Gc = take(size_t(n) * ld * 4);
  L.J = take(size_t(round_up16(n)) * ld * jsz);
  L.b = take(ld * 4);
  L.z = take(ld * 4);
  L.rs = take(ld * 4);
  L.R = take(ld * 4);
  L.sig = take(ld);
  L.c = take(size_t(P) * ld * 4);
  L.c2 = take(size_t(P) * ld * 4);
  L.e = take(size_t(P) * ld * 4);
  L.xb = take(xbits_words(int(ld), P) * 4);
  L.xb2 = take(xbits_words(int(ld), P) * 4);
  L.sig_all = take(size_t(P) * n);
  L.hpart = take(size_t(P) * n * 8);
  L.jw = take(bjac_words(int(ld)) * 4);
  L.A = take(size_t(m) * n * 4);
  L.y = take(size_t(m) * 4);
  L.total = o;
  return L;
}

// Arena head: device tables of one tick, per-slot stats, Cholesky scratch.
struct HeadLayout {
  size_t insts, rinsts, tiles, rowp, stp, stats, chol, total;
  int max_tiles;
};

HeadLayout head_layout(int max_slots, int max_n, bool chol) {
  HeadLayout H;
  H.max_tiles = max_slots * ((max_n + 15) / 16);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  H.insts = take(size_t(max_slots) * sizeof(BInst));
  H.rinsts = take(size_t(max_slots) * sizeof(BInst));
  H.tiles = take(size_t(H.max_tiles) * sizeof(BTile));
  H.rowp = take(size_t(max_slots + 1) * sizeof(int64_t));
  H.stp = take(size_t(max_slots + 1) * sizeof(int64_t));
  H.stats = take(size_t(max_slots) * sizeof(l0cim_stats));
  H.chol = take(chol ? chol_ws_bytes(max_n) : 0);
  H.total = o;
  return H;
}

struct Req {
  int64_t tag;
  int m, n;
  const float* A;
  int64_t lda;
  const float* y;
  uint64_t seed;
  float* R_out;
  uint8_t* sig_out;
  l0cim_stats* st_out;
  double t_submit, t_admit;
  size_t off, bytes, cost;   // cost: couplings bytes streamed per Euler step
  int slot, alt;
};

}  // namespace

struct l0cim_server_s {
  l0cim_cim_params cim;
  l0cim_solve_params sp;
  l0cim_dtype jdt;
  int P, qb, max_slots, max_n, cu_count;
  char* arena;
  size_t arena_bytes, heap0;
  HeadLayout head;
  hipStream_t stream;
  ServeSched<Req> q;                      // heap, slots, queue, admission, retirement
  std::vector<l0cim_completion> done;
  void* staging = nullptr;
  size_t staging_bytes = 0;
  hipEvent_t tick_done = nullptr;
  std::chrono::steady_clock::time_point t0;
  int64_t ticks = 0;
  bool broken = false;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  double eta_of(int alt) const {
    const double v = sp.eta_init * (1.0 - double(alt) / double(sp.velo));
    return v > sp.eta_end ? v : sp.eta_end;
  }

  l0cim_stats* slot_stats(int slot) const {
    return reinterpret_cast<l0cim_stats*>(arena + head.stats) + slot;
  }

  BInst make_inst(const Req& r) const {
    const ReqLayout L = req_layout(r.m, r.n, P, dtype_size(jdt));
    char* b = arena + r.off;
    BInst I{};
    I.n = r.n;
    I.m = r.m;
    I.ld = round_up32(r.n);
    I.ldj = I.ld;
    I.lda = r.n;
    I.alt = r.alt;
    I.seed = r.seed;
    I.eta = eta_of(r.alt);
    I.A = reinterpret_cast<const float*>(b + L.A);
    I.y = reinterpret_cast<const float*>(b + L.y);
    I.G = reinterpret_cast<float*>(b + L.G);
    I.Gc = reinterpret_cast<float*>(b + L.Gc);
    I.J = b + L.J;
    I.b = reinterpret_cast<float*>(b + L.b);
    I.z = reinterpret_cast<float*>(b + L.z);
    I.rs = reinterpret_cast<float*>(b + L.rs);
    I.R = reinterpret_cast<float*>(b + L.R);
    I.sig = reinterpret_cast<uint8_t*>(b + L.sig);
    I.c = reinterpret_cast<float*>(b + L.c);
    I.c2 = reinterpret_cast<float*>(b + L.c2);
    I.e = reinterpret_cast<float*>(b + L.e);
    I.xb = reinterpret_cast<uint32_t*>(b + L.xb);
    I.xb2 = reinterpret_cast<uint32_t*>(b + L.xb2);
    I.sig_all = reinterpret_cast<uint8_t*>(b + L.sig_all);
    I.hpart = reinterpret_cast<double*>(b + L.hpart);
    I.jw = reinterpret_cast<float*>(b + L.jw);
    I.st = slot_stats(r.slot);
    I.status = &I.st->status_bits;
    return I;
  }
};

namespace {

#define L0_TRY(x)                  \
  do {                             \
    l0cim_status _s = (x);         \
    if (_s != L0CIM_OK) return _s; \
  } while (0)

l0cim_status admit(l0cim_server_s* sv, Req& r, hipStream_t s) {
  const ReqLayout L = req_layout(r.m, r.n, sv->P, dtype_size(sv->jdt));
  char* b = sv->arena + r.off;
  L0_HIP(hipMemcpy2DAsync(b + L.A, size_t(r.n) * 4, r.A, size_t(r.lda) * 4, size_t(r.n) * 4, size_t(r.m),
                          hipMemcpyDeviceToDevice, s));
  L0_HIP(hipMemcpyAsync(b + L.y, r.y, size_t(r.m) * 4, hipMemcpyDeviceToDevice, s));
  L0_HIP(hipMemsetAsync(sv->slot_stats(r.slot), 0, sizeof(l0cim_stats), s));
  const BInst I = sv->make_inst(r);
  L0_TRY(launch_gram(L0CIM_F32, I.m, I.n, I.A, I.lda, I.y, I.G, I.ld, I.b, s));
  L0_TRY(launch_r_init(L0CIM_F32, I.n, I.G, I.ld, I.b, nullptr, I.R, I.status, s));
  return L0CIM_OK;
}

// One alternation of every resident request, then the report of those that
// are done.  Returns after the tick's device work has finished.
l0cim_status tick(l0cim_server_s* sv, int* n_done) {
  hipStream_t s = sv->stream;
  const double t_start = sv->now();
  // admission: arrival order, stop at the first request that does not fit
  // (in memory, or in the step budget unless nothing is resident)
  const int added = sv->q.admit(t_start);
  for (size_t k = sv->q.active.size() - size_t(added); k < sv->q.active.size(); ++k)
    L0_TRY(admit(sv, sv->q.active[k], s));
  *n_done = 0;
  if (sv->q.active.empty()) return L0CIM_OK;
  const int count = int(sv->q.active.size());
  // tile shape: the largest row block that still gives every CU four tiles
  auto tiles_for = [&](int rb) {
    int64_t t = 0;
    for (const Req& r : sv->q.active) t += (r.n + 16 * rb - 1) / (16 * rb);
    return t;
  };
  int rb = 1;
  for (int cand : {8, 4, 2})
    if (step_shape_ok(sv->qb, cand) && tiles_for(cand) >= 4 * sv->cu_count) {
      rb = cand;
      break;
    }
  const int tr = 16 * rb;
  // host tables in the pinned staging buffer (the previous tick has finished)
  char* h = static_cast<char*>(sv->staging);
  BInst* hi = reinterpret_cast<BInst*>(h);
  BInst* hr = reinterpret_cast<BInst*>(h + (sv->head.rinsts - sv->head.insts));
  BTile* ht = reinterpret_cast<BTile*>(h + (sv->head.tiles - sv->head.insts));
  int64_t* hrow = reinterpret_cast<int64_t*>(h + (sv->head.rowp - sv->head.insts));
  int64_t* hst = reinterpret_cast<int64_t*>(h + (sv->head.stp - sv->head.insts));
  std::vector<int> order(count);
  for (int k = 0; k < count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return sv->q.active[x].n > sv->q.active[y].n; });
  int nt = 0;
  hrow[0] = 0;
  hst[0] = 0;
  for (int k = 0; k < count; ++k) {
    const Req& r = sv->q.active[k];
    hi[k] = sv->make_inst(r);
    hrow[k + 1] = hrow[k] + round_up16(r.n);
    hst[k + 1] = hst[k] + int64_t(sv->P) * hi[k].ld;
  }
  for (int k : order) {
    hi[k].tile0 = nt;
    for (int r0 = 0; r0 < hi[k].n; r0 += tr) ht[nt++] = BTile{k, r0};
    hi[k].ntiles = nt - hi[k].tile0;
  }
  int nret = 0;
  for (int k = 0; k < count; ++k)
    if (sv->q.finishing(sv->q.active[k])) hr[nret++] = hi[k];
  // the staging buffer mirrors the head layout from the instance table on
  BatchDev d{};
  d.count = count;
  d.insts = reinterpret_cast<const BInst*>(sv->arena + sv->head.insts);
  d.tiles = reinterpret_cast<const BTile*>(sv->arena + sv->head.tiles);
  d.row_prefix = reinterpret_cast<const int64_t*>(sv->arena + sv->head.rowp);
  d.st_prefix = reinterpret_cast<const int64_t*>(sv->arena + sv->head.stp);
  d.eta = nullptr;
  L0_HIP(hipMemcpyAsync(sv->arena + sv->head.insts, h, sv->head.stats - sv->head.insts, hipMemcpyHostToDevice, s));
  // one alternation
  L0_TRY(launch_bcouplings(d, sv->jdt, hrow[count], s));
  L0_TRY(launch_binit(d, sv->P, -1, sv->cim.c0_std, hst[count], s));
  if (sv->cim.field == L0CIM_FIELD_BN) L0_TRY(launch_bbits(d, sv->qb, hst[count] / 32, s));
  const StepKernel fn = batch_step_kernel(sv->jdt, sv->cim.field, sv->qb, rb);
  if (!fn.fn) return set_error(L0CIM_ERR_UNSUPPORTED, "server: no step kernel for this shape");
  BStepArgs a{};
  a.P = sv->P;
  a.n_steps = sv->cim.n_steps;
  a.linear_j = sv->cim.linear_j;
  a.field = sv->cim.field;
  a.dt = sv->cim.dt;
  a.p_thr = sv->cim.p_thr;
  a.d = sv->cim.d;
  a.t_c = sv->cim.t_c;
  a.t_w = sv->cim.t_w;
  a.K = sv->cim.K;
  a.j = sv->cim.j;
  a.beta = sv->cim.beta;
  a.tau = sv->cim.tau;
  {
    ProfileScope prof(s);
    L0_TRY(enqueue_bsteps(d, fn, a, nt, 0, sv->cim.n_steps, s));
  }
  L0_TRY(launch_bselect(d, sv->P, s));
  L0_TRY(launch_bjacobi(d, nt, tr, sv->sp.dtc, sv->sp.cdp_iters, s));
  // report the requests that are done
  if (nret) {
    BatchDev dr{};
    dr.count = nret;
    dr.insts = reinterpret_cast<const BInst*>(sv->arena + sv->head.rinsts);
    if (sv->sp.final_refit_f64) {
      for (int k = 0; k < nret; ++k)
        L0_TRY(launch_chol_refit_a(L0CIM_F32, hr[k].m, hr[k].n, hr[k].A, hr[k].lda, hr[k].y, hr[k].sig, hr[k].R,
                                   hr[k].status, sv->arena + sv->head.chol, chol_ws_bytes(sv->max_n), s));
    }
    L0_TRY(launch_bobjective(dr, -1.0, sv->cim.n_steps, 0, sv->P, s));
    for (const Req& r : sv->q.active) {
      if (!sv->q.finishing(r)) continue;
      const BInst I = sv->make_inst(r);
      L0_HIP(hipMemcpyAsync(r.R_out, I.R, size_t(r.n) * 4, hipMemcpyDeviceToDevice, s));
      L0_HIP(hipMemcpyAsync(r.sig_out, I.sig, size_t(r.n), hipMemcpyDeviceToDevice, s));
      L0_HIP(hipMemcpyAsync(r.st_out, I.st, sizeof(l0cim_stats), hipMemcpyDeviceToDevice, s));
    }
  }
  L0_HIP(hipEventRecord(sv->tick_done, s));
  L0_HIP(hipEventSynchronize(sv->tick_done));
  const double t_end = sv->now();
  std::vector<Req> fin;
  sv->q.retire(fin);
  for (const Req& r : fin) {
    l0cim_completion c{};
    c.tag = r.tag;
    c.n = r.n;
    c.m = r.m;
    c.t_submit = r.t_submit;
    c.t_admit = r.t_admit;
    c.t_finish = t_end;
    sv->done.push_back(c);
  }
  *n_done = int(fin.size());
  ++sv->ticks;
  return L0CIM_OK;
}

}  // namespace

extern "C" {

size_t l0cim_server_request_bytes(int32_t m, int32_t n, const l0cim_solve_params* sp) {
  if (!sp || m <= 0 || n <= 0 || sp->replicas < 1) return 0;
  return req_layout(m, n, sp->replicas, dtype_size(l0cim_dtype(sp->j_dtype))).total;
}

size_t l0cim_server_arena_overhead(int32_t max_slots, int32_t max_n, const l0cim_solve_params* sp) {
  if (!sp || max_slots <= 0 || max_n <= 0) return 0;
  return head_layout(max_slots, max_n, sp->final_refit_f64 != 0).total;
}

l0cim_status l0cim_server_create(const l0cim_cim_params* cim, const l0cim_solve_params* sp, int32_t max_slots,
                                 int32_t max_n, void* arena, size_t arena_bytes, void* stream, l0cim_server* out) {
  if (!cim || !sp || !out || !arena) return set_error(L0CIM_ERR_ARG, "server_create: NULL pointer");
  if (max_slots < 1 || max_slots > 4096) return set_error(L0CIM_ERR_ARG, "server_create: max_slots must be 1..4096");
  if (max_n < 1 || max_n > 12288) return set_error(L0CIM_ERR_SHAPE, "server_create: max_n must be 1..12288");
  if (cim->n_steps < 0 || !(cim->dt > 0) || !(cim->tau > 0) || !(cim->t_w > 0) ||
      (cim->field != L0CIM_FIELD_CN && cim->field != L0CIM_FIELD_BN))
    return set_error(L0CIM_ERR_ARG, "server_create: invalid CIM parameters");
  if (sp->replicas < 1 || sp->replicas > 64) return set_error(L0CIM_ERR_ARG, "server_create: replicas must be 1..64");
  if (sp->n_outer <= 0 || sp->n_outer >= (1 << 24) || sp->velo <= 0 || sp->cdp_iters < 0)
    return set_error(L0CIM_ERR_ARG, "server_create: invalid outer schedule");
  if (sp->cdp != L0CIM_CDP_JACOBI) return set_error(L0CIM_ERR_UNSUPPORTED, "server: CDP is Jacobi");
  const l0cim_dtype jdt = l0cim_dtype(sp->j_dtype);
  if (jdt != L0CIM_F32 && jdt != L0CIM_BF16 && jdt != L0CIM_FP8E4M3)
    return set_error(L0CIM_ERR_UNSUPPORTED, "server couplings: F32, BF16 or FP8E4M3");
  if (reinterpret_cast<uintptr_t>(arena) % kAlign != 0)
    return set_error(L0CIM_ERR_ARG, "server_create: arena must be %zu-byte aligned", kAlign);
  const HeadLayout H = head_layout(max_slots, max_n, sp->final_refit_f64 != 0);
  if (arena_bytes < H.total + kAlign)
    return set_error(L0CIM_ERR_WORKSPACE, "server_create: arena needs more than %zu bytes", H.total);
  DeviceInfo dev;
  l0cim_status st = device_info(&dev);
  if (st != L0CIM_OK) return st;
  auto* sv = new l0cim_server_s();
  sv->cim = *cim;
  sv->sp = *sp;
  sv->jdt = jdt;
  sv->P = sp->replicas;
  sv->qb = sv->P <= 16 ? 1 : (sv->P <= 32 ? 2 : 4);
  sv->max_slots = max_slots;
  sv->max_n = max_n;
  sv->cu_count = dev.cu_count;
  sv->arena = static_cast<char*>(arena);
  sv->arena_bytes = arena_bytes;
  sv->head = H;
  sv->heap0 = H.total;
  sv->stream = static_cast<hipStream_t>(stream);
  const size_t heap = (arena_bytes - H.total) / kAlign * kAlign;
  sv->q.init(max_slots, H.total, heap, sp->n_outer);
  sv->staging_bytes = H.stats - H.insts;
  hipError_t he = hipHostMalloc(&sv->staging, sv->staging_bytes, hipHostMallocDefault);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&sv->tick_done, hipEventDisableTiming);
  if (he != hipSuccess) {
    if (sv->staging) (void)hipHostFree(sv->staging);
    delete sv;
    return hip_fail(he, "server_create");
  }
  sv->t0 = std::chrono::steady_clock::now();
  *out = sv;
  return L0CIM_OK;
}

double l0cim_server_clock(l0cim_server sv) { return sv ? sv->now() : 0.0; }

l0cim_status l0cim_server_submit(l0cim_server sv, int32_t m, int32_t n, const float* A, int64_t lda,
                                 const float* y, uint64_t seed, int64_t tag, float* R_out, uint8_t* sigma_out,
                                 l0cim_stats* stats_out) {
  if (!sv) return set_error(L0CIM_ERR_ARG, "server_submit: NULL server");
  if (sv->broken) return set_error(L0CIM_ERR_HIP, "server_submit: server stopped after a device error");
  if (!A || !y || !R_out || !sigma_out || !stats_out) return set_error(L0CIM_ERR_ARG, "server_submit: NULL pointer");
  if (m <= 0 || n <= 0 || lda < n) return set_error(L0CIM_ERR_SHAPE, "server_submit: bad shape");
  if (n > sv->max_n) return set_error(L0CIM_ERR_SHAPE, "server_submit: n = %d above the server's %d", n, sv->max_n);
  if (sv->sp.final_refit_f64 && chol_a_ws_bytes(n, m) > chol_ws_bytes(sv->max_n))
    return set_error(L0CIM_ERR_SHAPE, "server_submit: m = %d too large for the FP64 refit scratch", m);
  Req r{};
  r.tag = tag;
  r.m = m;
  r.n = n;
  r.A = A;
  r.lda = lda;
  r.y = y;
  r.seed = seed;
  r.R_out = R_out;
  r.sig_out = sigma_out;
  r.st_out = stats_out;
  r.bytes = req_layout(m, n, sv->P, dtype_size(sv->jdt)).total;
  r.cost = size_t(round_up16(n)) * size_t(round_up32(n)) * dtype_size(sv->jdt);
  if (r.bytes > sv->arena_bytes - sv->heap0)
    return set_error(L0CIM_ERR_WORKSPACE, "server_submit: request needs %zu bytes, the arena holds %zu", r.bytes,
                     sv->arena_bytes - sv->heap0);
  r.t_submit = sv->now();
  r.slot = -1;
  sv->q.pending.push_back(r);
  return L0CIM_OK;
}

l0cim_status l0cim_server_set_step_budget(l0cim_server sv, size_t bytes) {
  if (!sv) return set_error(L0CIM_ERR_ARG, "server_set_step_budget: NULL server");
  sv->q.step_budget = bytes;
  return L0CIM_OK;
}

l0cim_status l0cim_server_step(l0cim_server sv, int32_t* completed) {
  if (!sv) return set_error(L0CIM_ERR_ARG, "server_step: NULL server");
  if (sv->broken) return set_error(L0CIM_ERR_HIP, "server_step: server stopped after a device error");
  int done = 0;
  l0cim_status st = tick(sv, &done);
  if (st != L0CIM_OK) sv->broken = true;
  if (completed) *completed = done;
  return st;
}

int32_t l0cim_server_completed(l0cim_server sv, l0cim_completion* out, int32_t max) {
  if (!sv || !out || max <= 0) return 0;
  const int n = int(std::min<size_t>(sv->done.size(), size_t(max)));
  std::copy(sv->done.begin(), sv->done.begin() + n, out);
  sv->done.erase(sv->done.begin(), sv->done.begin() + n);
  return n;
}

l0cim_status l0cim_server_info(l0cim_server sv, int32_t* active, int32_t* pending, size_t* bytes_in_use,
                               size_t* heap_bytes, int64_t* ticks) {
  if (!sv) return set_error(L0CIM_ERR_ARG, "server_info: NULL server");
  if (active) *active = int32_t(sv->q.active.size());
  if (pending) *pending = int32_t(sv->q.pending.size());
  if (bytes_in_use) *bytes_in_use = sv->q.in_use;
  if (heap_bytes) *heap_bytes = (sv->arena_bytes - sv->heap0) / kAlign * kAlign;
  if (ticks) *ticks = sv->ticks;
  return L0CIM_OK;
}

l0cim_status l0cim_server_destroy(l0cim_server sv) {
  if (!sv) return L0CIM_OK;
  if (sv->tick_done) {
    (void)hipEventSynchronize(sv->tick_done);
    (void)hipEventDestroy(sv->tick_done);
  }
  if (sv->staging) (void)hipHostFree(sv->staging);
  delete sv;
  return L0CIM_OK;
}

}  // extern "C"

// ---- the scheduler alone: admission, slots and heap with no device -------

namespace {

struct SimReq {
  int64_t tag;
  int m, n;
  size_t bytes, cost, off;
  int slot, alt;
  double t_submit, t_admit;
};

}  // namespace

struct l0cim_server_sim_s {
  l0cim_solve_params sp;
  size_t jsz;
  int P, max_n;
  size_t heap0;
  ServeSched<SimReq> q;
  std::vector<l0cim_completion> done;
};

extern "C" {

l0cim_status l0cim_server_sim_create(const l0cim_solve_params* sp, int32_t max_slots, int32_t max_n,
                                     size_t arena_bytes, l0cim_server_sim* out) {
  if (!sp || !out) return set_error(L0CIM_ERR_ARG, "server_sim_create: NULL pointer");
  if (max_slots < 1 || max_slots > 4096) return set_error(L0CIM_ERR_ARG, "server_sim_create: max_slots must be 1..4096");
  if (max_n < 1 || max_n > 12288) return set_error(L0CIM_ERR_SHAPE, "server_sim_create: max_n must be 1..12288");
  if (sp->replicas < 1 || sp->replicas > 64 || sp->n_outer <= 0 || sp->n_outer >= (1 << 24))
    return set_error(L0CIM_ERR_ARG, "server_sim_create: replicas 1..64 and a positive n_outer");
  const l0cim_dtype jdt = l0cim_dtype(sp->j_dtype);
  if (jdt != L0CIM_F32 && jdt != L0CIM_BF16 && jdt != L0CIM_FP8E4M3)
    return set_error(L0CIM_ERR_UNSUPPORTED, "server couplings: F32, BF16 or FP8E4M3");
  const HeadLayout H = head_layout(max_slots, max_n, sp->final_refit_f64 != 0);
  if (arena_bytes < H.total + kAlign)
    return set_error(L0CIM_ERR_WORKSPACE, "server_sim_create: arena needs more than %zu bytes", H.total);
  auto* sim = new l0cim_server_sim_s();
  sim->sp = *sp;
  sim->jsz = dtype_size(jdt);
  sim->P = sp->replicas;
  sim->max_n = max_n;
  sim->heap0 = H.total;
  sim->q.init(max_slots, H.total, (arena_bytes - H.total) / kAlign * kAlign, sp->n_outer);
  *out = sim;
  return L0CIM_OK;
}

l0cim_status l0cim_server_sim_submit(l0cim_server_sim sim, int32_t m, int32_t n, int64_t tag, double t_submit) {
  if (!sim) return set_error(L0CIM_ERR_ARG, "server_sim_submit: NULL simulation");
  if (m <= 0 || n <= 0) return set_error(L0CIM_ERR_SHAPE, "server_sim_submit: bad shape");
  if (n > sim->max_n) return set_error(L0CIM_ERR_SHAPE, "server_sim_submit: n = %d above %d", n, sim->max_n);
  if (sim->sp.final_refit_f64 && chol_a_ws_bytes(n, m) > chol_ws_bytes(sim->max_n))
    return set_error(L0CIM_ERR_SHAPE, "server_sim_submit: m = %d too large for the FP64 refit scratch", m);
  SimReq r{};
  r.tag = tag;
  r.m = m;
  r.n = n;
  r.bytes = req_layout(m, n, sim->P, sim->jsz).total;
  r.cost = size_t(round_up16(n)) * size_t(round_up32(n)) * sim->jsz;
  if (r.bytes > sim->q.heap_bytes)
    return set_error(L0CIM_ERR_WORKSPACE, "server_sim_submit: request needs %zu bytes, the arena holds %zu", r.bytes,
                     sim->q.heap_bytes);
  r.slot = -1;
  r.t_submit = t_submit;
  sim->q.pending.push_back(r);
  return L0CIM_OK;
}

l0cim_status l0cim_server_sim_set_step_budget(l0cim_server_sim sim, size_t bytes) {
  if (!sim) return set_error(L0CIM_ERR_ARG, "server_sim_set_step_budget: NULL simulation");
  sim->q.step_budget = bytes;
  return L0CIM_OK;
}

l0cim_status l0cim_server_sim_tick(l0cim_server_sim sim, double t_start, double t_end, int32_t* admitted,
                                   int32_t* completed) {
  if (!sim) return set_error(L0CIM_ERR_ARG, "server_sim_tick: NULL simulation");
  const int added = sim->q.admit(t_start);
  std::vector<SimReq> fin;
  if (!sim->q.active.empty()) sim->q.retire(fin);
  for (const SimReq& r : fin) {
    l0cim_completion c{};
    c.tag = r.tag;
    c.n = r.n;
    c.m = r.m;
    c.t_submit = r.t_submit;
    c.t_admit = r.t_admit;
    c.t_finish = t_end;
    sim->done.push_back(c);
  }
  if (admitted) *admitted = added;
  if (completed) *completed = int32_t(fin.size());
  return L0CIM_OK;
}

int32_t l0cim_server_sim_completed(l0cim_server_sim sim, l0cim_completion* out, int32_t max) {
  if (!sim || !out || max <= 0) return 0;
  const int n = int(std::min<size_t>(sim->done.size(), size_t(max)));
  std::copy(sim->done.begin(), sim->done.begin() + n, out);
  sim->done.erase(sim->done.begin(), sim->done.begin() + n);
  return n;
}

int32_t l0cim_server_sim_resident(l0cim_server_sim sim, int64_t* tags, int32_t* slots, size_t* offsets,
                                  int32_t* alternations, int32_t max) {
  if (!sim) return 0;
  const int n = int(std::min<size_t>(sim->q.active.size(), size_t(max > 0 ? max : 0)));
  for (int k = 0; k < n; ++k) {
    const SimReq& r = sim->q.active[k];
    if (tags) tags[k] = r.tag;
    if (slots) slots[k] = r.slot;
    if (offsets) offsets[k] = r.off - sim->heap0;
    if (alternations) alternations[k] = r.alt;
  }
  return int32_t(sim->q.active.size());
}

l0cim_status l0cim_server_sim_info(l0cim_server_sim sim, int32_t* active, int32_t* pending, size_t* bytes_in_use,
                                   size_t* heap_bytes, int32_t* free_blocks) {
  if (!sim) return set_error(L0CIM_ERR_ARG, "server_sim_info: NULL simulation");
  if (active) *active = int32_t(sim->q.active.size());
  if (pending) *pending = int32_t(sim->q.pending.size());
  if (bytes_in_use) *bytes_in_use = sim->q.in_use;
  if (heap_bytes) *heap_bytes = sim->q.heap_bytes;
  if (free_blocks) *free_blocks = int32_t(sim->q.free_blocks.size());
  return L0CIM_OK;
}

l0cim_status l0cim_server_sim_destroy(l0cim_server_sim sim) {
  delete sim;
  return L0CIM_OK;
}

}  // extern "C"
