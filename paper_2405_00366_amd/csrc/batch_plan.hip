// Host side of the batched engine: the plan (pool layout, row-tile table,
// tile shape picked by timing the candidates once per shape class), the HIP
// graph of one CIM run, and the C entry points.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batch.h"

using namespace l0;

// Where one instance lives: element offsets into the plan's pools (G, J,
// per-spin vectors, state, supports) and into the caller's pools (A, y, R, sigma).
struct PoolSlot {
  int n, m, ld, lda;
  int64_t oG, oJ, oV, oS, oSig, oX, oA, oY, oW, oB;
  uint64_t seed;
};

struct l0cim_batch_plan_s {
  int count = 0, P = 1, qb = 1;
  l0cim_cim_params cim;
  l0cim_solve_params sp;
  l0cim_dtype jdt = L0CIM_F32;
  std::vector<l0cim_instance> inst;
  std::vector<PoolSlot> base;
  std::vector<int64_t> row_prefix, st_prefix;
  int64_t nG = 0, nJ = 0, nV = 0, nS = 0, nSig = 0, nW = 0, nB = 0, max_tiles = 0;
  int max_ld = 0, max_n = 0, max_m = 0;
  struct {
    size_t insts, tiles, rowp, stp, eta, G, Gc, b, z, rs, J, c, c2, e, xb, xb2, sig, hpart, jw, chol, total;
  } off{};
  int rb = 0;
  bool tuned = false;
  std::string key;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* graph_ws = nullptr;
  int graph_rb = 0;
  // workspace and tile count of the solve opened by l0cim_batch_begin
  const void* open_ws = nullptr;
  int open_ntiles = 0;
  // pinned staging buffer of the device tables; an upload waits for the
  // previous one to have left it before writing it again
  void* staging = nullptr;
  size_t staging_bytes = 0;
  hipEvent_t staged = nullptr;
};

namespace {

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;   // shape class -> rows per wavefront block count

int round_up_i(int x, int a) { return (x + a - 1) / a * a; }

// Row tiles of every instance.  The dispatcher deals workgroup b to XCD
// b mod 8, and each XCD has its own L2, so the instances are spread over the
// XCDs whole (largest first, each to the XCD with the least coupling bytes so
// far): the amplitudes of an instance are then fetched into one L2 rather
// than eight.  Workgroup b = 8 i + x takes tile i of XCD x's list (largest
// work first, so that the tail of a step is made of small tiles); shorter
// lists are padded with empty tiles (inst = -1), which exit at once.  Results
// do not depend on the order: every output row is computed by one wavefront
// in a fixed k order.
void tile_table(const l0cim_batch_plan_s* p, int rb, std::vector<BTile>& tiles) {
  const int tr = 16 * rb;
  std::vector<int> order(p->count);
  for (int k = 0; k < p->count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p->base[x].n > p->base[y].n; });
  std::vector<BTile> bins[kXcds];
  double load[kXcds] = {};
  for (int k : order) {
    int x = 0;
    for (int j = 1; j < kXcds; ++j)
      if (load[j] < load[x]) x = j;
    load[x] += double(round_up_i(p->base[k].n, tr)) * p->base[k].ld;
    for (int r0 = 0; r0 < p->base[k].n; r0 += tr) bins[x].push_back(BTile{k, r0});
  }
  size_t len = 0;
  for (auto& b : bins) len = b.size() > len ? b.size() : len;
  tiles.clear();
  for (size_t i = 0; i < len; ++i)
    for (auto& b : bins) tiles.push_back(i < b.size() ? b[i] : BTile{-1, 0});
}

struct Pools {
  char* ws;
  const float *A, *y;
  float* R;
  uint8_t* sig;
  l0cim_stats* stats;
};

BInst make_inst(const l0cim_batch_plan_s* p, int k, const Pools& pl) {
  const PoolSlot& q = p->base[k];
  char* b = pl.ws;
  BInst I{};
  I.n = q.n;
  I.m = q.m;
  I.ld = q.ld;
  I.ldj = q.ld;
  I.lda = q.lda;
  I.seed = q.seed;
  I.A = pl.A + q.oA;
  I.y = pl.y + q.oY;
  I.G = reinterpret_cast<float*>(b + p->off.G) + q.oG;
  I.Gc = reinterpret_cast<float*>(b + p->off.Gc) + q.oG;
  I.J = b + p->off.J + size_t(q.oJ) * dtype_size(p->jdt);
  I.b = reinterpret_cast<float*>(b + p->off.b) + q.oV;
  I.z = reinterpret_cast<float*>(b + p->off.z) + q.oV;
  I.rs = reinterpret_cast<float*>(b + p->off.rs) + q.oV;
  I.R = pl.R + q.oX;
  I.sig = pl.sig + q.oX;
  I.c = reinterpret_cast<float*>(b + p->off.c) + q.oS;
  I.c2 = reinterpret_cast<float*>(b + p->off.c2) + q.oS;
  I.e = reinterpret_cast<float*>(b + p->off.e) + q.oS;
  I.xb = reinterpret_cast<uint32_t*>(b + p->off.xb) + q.oB;
  I.xb2 = reinterpret_cast<uint32_t*>(b + p->off.xb2) + q.oB;
  I.sig_all = reinterpret_cast<uint8_t*>(b + p->off.sig) + q.oSig;
  I.jw = reinterpret_cast<float*>(b + p->off.jw) + q.oW;
  I.hpart = reinterpret_cast<double*>(b + p->off.hpart) + q.oSig;
  I.st = pl.stats + k;
  I.status = &pl.stats[k].status_bits;
  return I;
}

BatchDev carve(const l0cim_batch_plan_s* p, char* ws) {
  BatchDev d;
  d.count = p->count;
  d.insts = reinterpret_cast<const BInst*>(ws + p->off.insts);
  d.tiles = reinterpret_cast<const BTile*>(ws + p->off.tiles);
  d.row_prefix = reinterpret_cast<const int64_t*>(ws + p->off.rowp);
  d.st_prefix = reinterpret_cast<const int64_t*>(ws + p->off.stp);
  d.eta = reinterpret_cast<const double*>(ws + p->off.eta);
  return d;
}

// Upload the instance table (with tile ranges for rows-per-block `rb`), the
// tile table and the prefix tables through the pinned staging buffer.
l0cim_status upload_tables(l0cim_batch_plan_s* p, const BatchDev& d, const Pools& pl, int rb, hipStream_t s,
                           int* ntiles) {
  std::vector<BTile> tiles;
  tile_table(p, rb, tiles);
  const size_t bi = size_t(p->count) * sizeof(BInst), bt = tiles.size() * sizeof(BTile);
  const size_t bp = size_t(p->count + 1) * sizeof(int64_t);
  L0_HIP(hipEventSynchronize(p->staged));
  char* h = static_cast<char*>(p->staging);
  BInst* hi = reinterpret_cast<BInst*>(h);
  for (int k = 0; k < p->count; ++k) hi[k] = make_inst(p, k, pl);
  for (size_t t = 0; t < tiles.size(); ++t) {
    if (tiles[t].inst < 0) continue;   // padding
    BInst& I = hi[tiles[t].inst];
    if (tiles[t].row0 == 0) {
      I.tile0 = int(t);
      I.ntiles = 0;
    }
    ++I.ntiles;
  }
  memcpy(h + align_up(bi), tiles.data(), bt);
  memcpy(h + align_up(bi) + align_up(bt), p->row_prefix.data(), bp);
  memcpy(h + align_up(bi) + align_up(bt) + align_up(bp), p->st_prefix.data(), bp);
  L0_HIP(hipMemcpyAsync(const_cast<BInst*>(d.insts), h, bi, hipMemcpyHostToDevice, s));
  L0_HIP(hipMemcpyAsync(const_cast<BTile*>(d.tiles), h + align_up(bi), bt, hipMemcpyHostToDevice, s));
  L0_HIP(hipMemcpyAsync(const_cast<int64_t*>(d.row_prefix), h + align_up(bi) + align_up(bt), bp,
                        hipMemcpyHostToDevice, s));
  L0_HIP(hipMemcpyAsync(const_cast<int64_t*>(d.st_prefix), h + align_up(bi) + align_up(bt) + align_up(bp), bp,
                        hipMemcpyHostToDevice, s));
  L0_HIP(hipEventRecord(p->staged, s));
  *ntiles = int(tiles.size());
  return L0CIM_OK;
}

BStepArgs step_args(const l0cim_batch_plan_s* p) {
  BStepArgs a;
  a.P = p->P;
  a.n_steps = p->cim.n_steps;
  a.linear_j = p->cim.linear_j;
  a.field = p->cim.field;
  a.dt = p->cim.dt;
  a.p_thr = p->cim.p_thr;
  a.d = p->cim.d;
  a.t_c = p->cim.t_c;
  a.t_w = p->cim.t_w;
  a.K = p->cim.K;
  a.j = p->cim.j;
  a.beta = p->cim.beta;
  a.tau = p->cim.tau;
  a.trace = nullptr;
  a.trace_steps = 0;
  return a;
}

// Enqueue Euler steps k0..k1 (inclusive) of one CIM run.
l0cim_status enqueue_steps(const l0cim_batch_plan_s* p, const BatchDev& d, int rb, int ntiles, int k0, int k1,
                           hipStream_t s) {
  const StepKernel fn = batch_step_kernel(p->jdt, p->cim.field, p->qb, rb);
  if (!fn.fn) return set_error(L0CIM_ERR_UNSUPPORTED, "batched step: no kernel for this shape");
  return enqueue_bsteps(d, fn, step_args(p), ntiles, k0, k1, s);
}

std::string shape_key(const l0cim_batch_plan_s* p) {
  double sum_n2 = 0;
  for (auto& i : p->inst) sum_n2 += double(i.n) * i.n;
  int b2 = 0;
  while ((1ull << b2) < uint64_t(sum_n2 + 1)) ++b2;
  int bc = 0;
  while ((1 << bc) < p->count) ++bc;
  char buf[128];
  snprintf(buf, sizeof(buf), "P%d/j%d/f%d/n2_%d/c%d/nmax%d", p->P, int(p->jdt), p->cim.field, b2, bc,
           round_up_i(p->max_n, 256));
  return buf;
}

// Time every candidate tile shape on the current problem; the state it
// leaves behind is discarded (every alternation starts from init_state).
l0cim_status autotune(l0cim_batch_plan_s* p, const BatchDev& d, const Pools& pl, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(p->key);
    if (it != g_tune.end()) {
      p->rb = it->second;
      p->tuned = true;
      return L0CIM_OK;
    }
  }
  int ntiles = 0;
  hipEvent_t e0, e1;
  L0_HIP(hipEventCreate(&e0));
  L0_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int best_rb = 2;
  const int steps = p->cim.n_steps > 0 ? (p->cim.n_steps < 8 ? p->cim.n_steps : 8) : 0;
  for (int rb : {1, 2, 4, 8}) {
    if (!step_shape_ok(p->qb, rb)) continue;
    l0cim_status st = upload_tables(p, d, pl, rb, s, &ntiles);
    if (st != L0CIM_OK) return st;
    if (steps == 0) break;
    st = enqueue_steps(p, d, rb, ntiles, 0, 1, s);
    if (st != L0CIM_OK) return st;
    L0_HIP(hipEventRecord(e0, s));
    st = enqueue_steps(p, d, rb, ntiles, 0, steps - 1, s);
    if (st != L0CIM_OK) return st;
    L0_HIP(hipEventRecord(e1, s));
    L0_HIP(hipEventSynchronize(e1));
    float ms = 0;
    L0_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      best_rb = rb;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->rb = best_rb;
  p->tuned = true;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[p->key] = best_rb;
  return L0CIM_OK;
}

}  // namespace

namespace {

double plan_eta(const l0cim_batch_plan_s* p, int i) {
  double v = p->sp.eta_init * (1.0 - double(i) / double(p->sp.velo));
  return v > p->sp.eta_end ? v : p->sp.eta_end;
}

l0cim_status check_solve_args(l0cim_batch_plan p, const float* A, const float* y, float* R, uint8_t* sigma,
                              l0cim_stats* stats, void* ws, size_t ws_bytes, const char* who) {
  if (!p) return set_error(L0CIM_ERR_ARG, "%s: NULL plan", who);
  if (!A || !y || !R || !sigma || !stats) return set_error(L0CIM_ERR_ARG, "%s: NULL pointer", who);
  if (!ws || ws_bytes < p->off.total)
    return set_error(L0CIM_ERR_WORKSPACE, "%s: workspace needs %zu bytes", who, p->off.total);
  return L0CIM_OK;
}

// The HIP graph of one CIM run (n_steps + 1 launches), rebuilt when the
// workspace or the tile shape changes.
l0cim_status ensure_graph(l0cim_batch_plan_s* p, const BatchDev& d, const void* ws, int ntiles) {
  if (p->graph_ws == ws && p->graph_rb == p->rb && p->exec) return L0CIM_OK;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->graph_ws = nullptr;
  if (!p->cap_stream) L0_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  L0_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  l0cim_status st = enqueue_steps(p, d, p->rb, ntiles, 0, p->cim.n_steps, p->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(p->cap_stream, &g);
  if (st != L0CIM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
  p->graph = g;
  L0_HIP(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
  p->graph_ws = ws;
  p->graph_rb = p->rb;
  return L0CIM_OK;
}

}  // namespace

extern "C" {

l0cim_status l0cim_batch_plan_create(int32_t count, const l0cim_instance* inst, const l0cim_cim_params* cim,
                                     const l0cim_solve_params* sp, l0cim_batch_plan* out) {
  if (!out || !inst || !cim || !sp) return set_error(L0CIM_ERR_ARG, "batch_plan_create: NULL pointer");
  if (count <= 0) return set_error(L0CIM_ERR_SHAPE, "batch_plan_create: count must be positive");
  if (cim->n_steps < 0 || !(cim->dt > 0) || !(cim->tau > 0) || !(cim->t_w > 0) ||
      (cim->field != L0CIM_FIELD_CN && cim->field != L0CIM_FIELD_BN))
    return set_error(L0CIM_ERR_ARG, "batch_plan_create: invalid CIM parameters");
  if (sp->replicas < 1 || sp->replicas > 64) return set_error(L0CIM_ERR_ARG, "batch_plan_create: replicas must be 1..64");
  if (sp->n_outer <= 0 || sp->n_outer >= (1 << 24) || sp->velo <= 0 || sp->cdp_iters < 0)
    return set_error(L0CIM_ERR_ARG, "batch_plan_create: invalid outer schedule");
  if (sp->cdp != L0CIM_CDP_JACOBI) return set_error(L0CIM_ERR_UNSUPPORTED, "batched CDP is Jacobi");
  const l0cim_dtype jdt = l0cim_dtype(sp->j_dtype);
  if (jdt != L0CIM_F32 && jdt != L0CIM_BF16 && jdt != L0CIM_FP8E4M3)
    return set_error(L0CIM_ERR_UNSUPPORTED, "batched couplings: F32, BF16 or FP8E4M3");
  auto* p = new l0cim_batch_plan_s();
  p->count = count;
  p->P = sp->replicas;
  p->qb = p->P <= 16 ? 1 : (p->P <= 32 ? 2 : 4);
  p->cim = *cim;
  p->sp = *sp;
  p->jdt = jdt;
  p->inst.assign(inst, inst + count);
  p->base.resize(count);
  p->row_prefix.assign(count + 1, 0);
  p->st_prefix.assign(count + 1, 0);
  const size_t jsz = dtype_size(jdt);
  for (int k = 0; k < count; ++k) {
    const l0cim_instance& I = inst[k];
    if (I.m <= 0 || I.n <= 0 || I.lda < I.n || I.n > 12288 || I.lda > (int64_t(1) << 31) ||
        I.a_offset < 0 || I.y_offset < 0 || I.x_offset < 0) {
      delete p;
      return set_error(L0CIM_ERR_SHAPE, "batch_plan_create: instance %d has a bad shape or offset", k);
    }
    PoolSlot b{};
    b.n = I.n;
    b.m = I.m;
    b.ld = round_up_i(I.n, 32);
    b.lda = int(I.lda);
    b.oG = p->nG;
    b.oJ = p->nJ;
    b.oV = p->nV;
    b.oS = p->nS;
    b.oSig = p->nSig;
    b.oW = p->nW;
    b.oB = p->nB;
    b.oX = I.x_offset;
    b.oA = I.a_offset;
    b.oY = I.y_offset;
    b.seed = I.seed;
    p->nG += int64_t(b.n) * b.ld;
    p->nJ += int64_t(round_up16(b.n)) * b.ld;
    p->nV += b.ld;
    p->nS += int64_t(p->P) * b.ld;
    p->nSig += int64_t(p->P) * b.n;
    p->nW += int64_t(bjac_words(b.ld));
    p->nB += int64_t(xbits_words(b.ld, p->P));
    p->max_tiles += (b.n + 15) / 16;
    p->max_ld = b.ld > p->max_ld ? b.ld : p->max_ld;
    p->max_n = b.n > p->max_n ? b.n : p->max_n;
    p->max_m = b.m > p->max_m ? b.m : p->max_m;
    p->row_prefix[k + 1] = p->row_prefix[k] + round_up16(b.n);
    p->st_prefix[k + 1] = p->st_prefix[k] + int64_t(p->P) * b.ld;
    p->base[k] = b;
  }
  p->max_tiles *= kXcds;   // room for the empty tiles that pad the XCD lists (tile_table)
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  p->off.insts = take(count * sizeof(BInst));
  p->off.tiles = take(size_t(p->max_tiles) * sizeof(BTile));
  p->off.rowp = take((count + 1) * sizeof(int64_t));
  p->off.stp = take((count + 1) * sizeof(int64_t));
  p->off.eta = take(sizeof(double));
  p->off.G = take(size_t(p->nG) * 4);
  p->off.Gc = take(size_t(p->nG) * 4);
  p->off.b = take(size_t(p->nV) * 4);
  p->off.z = take(size_t(p->nV) * 4);
  p->off.rs = take(size_t(p->nV) * 4);
  p->off.J = take(size_t(p->nJ) * jsz);
  p->off.c = take(size_t(p->nS) * 4);
  p->off.c2 = take(size_t(p->nS) * 4);
  p->off.e = take(size_t(p->nS) * 4);
  p->off.xb = take(size_t(p->nB) * 4);
  p->off.xb2 = take(size_t(p->nB) * 4);
  p->off.sig = take(size_t(p->nSig));
  p->off.hpart = take(size_t(p->nSig) * sizeof(double));
  p->off.jw = take(size_t(p->nW) * 4);
  p->off.chol = take(sp->final_refit_f64 ? chol_a_ws_bytes(p->max_n, p->max_m) : 0);
  p->off.total = o;
  p->key = shape_key(p);
  p->staging_bytes = align_up(count * sizeof(BInst)) + align_up(size_t(p->max_tiles) * sizeof(BTile)) +
                     2 * align_up((count + 1) * sizeof(int64_t));
  hipError_t he = hipHostMalloc(&p->staging, p->staging_bytes, hipHostMallocDefault);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
  if (he != hipSuccess) {
    if (p->staging) (void)hipHostFree(p->staging);
    delete p;
    return hip_fail(he, "batch_plan_create: staging buffer");
  }
  *out = p;
  return L0CIM_OK;
}

size_t l0cim_batch_plan_workspace_bytes(l0cim_batch_plan plan) { return plan ? plan->off.total : 0; }

l0cim_status l0cim_batch_plan_info(l0cim_batch_plan plan, int32_t* rows_per_tile, int32_t* tiles,
                                   int32_t* tuned) {
  if (!plan) return set_error(L0CIM_ERR_ARG, "batch_plan_info: NULL plan");
  int rb = plan->rb ? plan->rb : 2;
  std::vector<BTile> t;
  tile_table(plan, rb, t);
  if (rows_per_tile) *rows_per_tile = 16 * rb;
  if (tiles) *tiles = int32_t(t.size());
  if (tuned) *tuned = plan->tuned ? 1 : 0;
  return L0CIM_OK;
}

l0cim_status l0cim_batch_plan_destroy(l0cim_batch_plan plan) {
  if (!plan) return L0CIM_OK;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  if (plan->staged) {
    (void)hipEventSynchronize(plan->staged);
    (void)hipEventDestroy(plan->staged);
  }
  if (plan->staging) (void)hipHostFree(plan->staging);
  delete plan;
  return L0CIM_OK;
}

l0cim_status l0cim_batch_begin(l0cim_batch_plan p, const float* A, const float* y, float* R, uint8_t* sigma,
                               l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  l0cim_status cs = check_solve_args(p, A, y, R, sigma, stats, ws, ws_bytes, "batch_begin");
  if (cs != L0CIM_OK) return cs;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  BatchDev d = carve(p, base);
  const Pools pl{base, A, y, R, sigma, stats};
#define L0_TRY(x)                  \
  do {                             \
    l0cim_status _s = (x);         \
    if (_s != L0CIM_OK) return _s; \
  } while (0)
  p->open_ws = nullptr;
  int ntiles = 0;
  L0_TRY(upload_tables(p, d, pl, p->rb ? p->rb : 2, s, &ntiles));
  L0_TRY(launch_bstats_init(d, s));
  for (int k = 0; k < p->count; ++k) {
    const BInst I = make_inst(p, k, pl);
    L0_TRY(launch_gram(L0CIM_F32, I.m, I.n, I.A, I.lda, I.y, I.G, I.ld, I.b, s));
    L0_TRY(launch_r_init(L0CIM_F32, I.n, I.G, I.ld, I.b, nullptr, I.R, I.status, s));
  }
  const int64_t total_rows = p->row_prefix[p->count];
  const int64_t total_state = p->st_prefix[p->count];
  if (!p->tuned) {
    // the candidate tiles are timed on the first alternation's state, which
    // the real first alternation rebuilds from scratch
    L0_TRY(launch_bset_scalar(const_cast<double*>(d.eta), p->sp.eta_init, s));
    L0_TRY(launch_bcouplings(d, p->jdt, total_rows, s));
    L0_TRY(launch_binit(d, p->P, 0, p->cim.c0_std, total_state, s));
    if (p->cim.field == L0CIM_FIELD_BN) L0_TRY(launch_bbits(d, p->qb, total_state / 32, s));
    L0_TRY(autotune(p, d, pl, s));
  }
  L0_TRY(upload_tables(p, d, pl, p->rb, s, &ntiles));
  p->open_ws = ws;
  p->open_ntiles = ntiles;
  return L0CIM_OK;
}

l0cim_status l0cim_batch_alternations(l0cim_batch_plan p, int32_t i0, int32_t i1, const float* A, const float* y,
                                      float* R, uint8_t* sigma, l0cim_stats* stats, void* ws, size_t ws_bytes,
                                      void* stream) {
  l0cim_status cs = check_solve_args(p, A, y, R, sigma, stats, ws, ws_bytes, "batch_alternations");
  if (cs != L0CIM_OK) return cs;
  if (p->open_ws != ws) return set_error(L0CIM_ERR_ARG, "batch_alternations: no batch_begin on this workspace");
  if (i0 < 0 || i1 < i0 || i1 > p->sp.n_outer)
    return set_error(L0CIM_ERR_ARG, "batch_alternations: range [%d, %d) outside [0, %d)", i0, i1, p->sp.n_outer);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  BatchDev d = carve(p, base);
  const int ntiles = p->open_ntiles;
  const int64_t total_rows = p->row_prefix[p->count];
  const int64_t total_state = p->st_prefix[p->count];
  const bool use_graph = p->cim.n_steps >= 16 && !(p->sp.flags & L0CIM_SOLVE_NO_GRAPH);
  if (use_graph && i1 > i0) L0_TRY(ensure_graph(p, d, ws, ntiles));
  for (int i = i0; i < i1; ++i) {
    L0_TRY(launch_bset_scalar(const_cast<double*>(d.eta), plan_eta(p, i), s));
    L0_TRY(launch_bcouplings(d, p->jdt, total_rows, s));
    L0_TRY(launch_binit(d, p->P, i, p->cim.c0_std, total_state, s));
    if (p->cim.field == L0CIM_FIELD_BN) L0_TRY(launch_bbits(d, p->qb, total_state / 32, s));
    {
      ProfileScope prof(s);
      if (use_graph) {
        L0_HIP(hipGraphLaunch(p->exec, s));
      } else {
        L0_TRY(enqueue_steps(p, d, p->rb, ntiles, 0, p->cim.n_steps, s));
      }
    }
    L0_TRY(launch_bselect(d, p->P, s));
    L0_TRY(launch_bjacobi(d, ntiles, 16 * p->rb, p->sp.dtc, p->sp.cdp_iters, s));
  }
  return L0CIM_OK;
}

l0cim_status l0cim_batch_finish(l0cim_batch_plan p, const float* A, const float* y, float* R, uint8_t* sigma,
                                l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  l0cim_status cs = check_solve_args(p, A, y, R, sigma, stats, ws, ws_bytes, "batch_finish");
  if (cs != L0CIM_OK) return cs;
  if (p->open_ws != ws) return set_error(L0CIM_ERR_ARG, "batch_finish: no batch_begin on this workspace");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  BatchDev d = carve(p, base);
  const Pools pl{base, A, y, R, sigma, stats};
  if (p->sp.final_refit_f64) {
    void* cws = base + p->off.chol;
    for (int k = 0; k < p->count; ++k) {
      const BInst I = make_inst(p, k, pl);
      L0_TRY(launch_chol_refit_a(L0CIM_F32, I.m, I.n, I.A, I.lda, I.y, I.sig, I.R, I.status, cws,
                                 chol_a_ws_bytes(p->max_n, p->max_m), s));
    }
  }
  const double eta = plan_eta(p, p->sp.n_outer - 1);
  L0_TRY(launch_bobjective(d, 0.5 * eta * eta, p->cim.n_steps, p->sp.n_outer, p->P, s));
  return L0CIM_OK;
}

l0cim_status l0cim_solve_batched(l0cim_batch_plan p, const float* A, const float* y, float* R, uint8_t* sigma,
                                 l0cim_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  L0_TRY(l0cim_batch_begin(p, A, y, R, sigma, stats, ws, ws_bytes, stream));
  L0_TRY(l0cim_batch_alternations(p, 0, p->sp.n_outer, A, y, R, sigma, stats, ws, ws_bytes, stream));
  L0_TRY(l0cim_batch_finish(p, A, y, R, sigma, stats, ws, ws_bytes, stream));
  return L0CIM_OK;
}
#undef L0_TRY

}  // extern "C"
