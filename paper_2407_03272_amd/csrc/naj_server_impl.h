// Serving loop: continuous batching of independent solve requests.
//
// Part of the naj_api.hip translation unit (it uses the system, pool and batch
// internals defined there); holds the naj_server_* entry points.
//
// A server owns one pool of device memory (its budget) and a table of slots.  A
// request is admitted into a free slot when its matrix, vectors and work items fit:
// its system is built on the server's admission stream, then a small kernel on the
// pass stream writes the slot's record, work items and control blocks, ordered after
// the build by an event.  The pass stream replays a captured chunk of batch passes
// (active-list rebuild, then graph_len item + decision kernel pairs) over every
// occupied slot; a request that arrives while others run joins at the next chunk,
// and a finished one gives back its slot and memory when its result is taken.
// Every request does the arithmetic of a batch of its own (its work items and
// summation orders depend only on its system), so its result does not depend on
// what else is being served.

struct naj_server {
  int device = 0;
  naj_opts opts;
  int max_slots = 0;
  int max_rhs = 0;
  int tile_cap = 0;
  hipStream_t st = nullptr;    // passes (the caller's stream)
  hipStream_t adm = nullptr;   // admission: system builds and uploads
  Pool pool;
  RangeAlloc items;            // ranges of the work-item table
  BatchSys* d_sys = nullptr;
  Ctrl* d_ctrl = nullptr;      // kMaxRhs per slot
  PassView* d_vt = nullptr;    // kMaxRhs per slot
  BatchTile* d_tiles = nullptr;
  int* d_active = nullptr;
  int* d_nactive = nullptr;
  int* d_sact = nullptr;
  int* d_nsact = nullptr;
  unsigned int* d_done = nullptr;
  int* d_slot_done = nullptr;
  static constexpr int kRing = 4;   // chunks in flight at most
  int* h_flags = nullptr;      // pinned, kRing x max_slots: slot_done after each chunk in flight
  Ctrl* h_ctrl = nullptr;      // pinned, kMaxRhs: a finished request's control blocks
  hipEvent_t evc[kRing] = {};
  hipEvent_t ev_adm = nullptr;
  int head = 0, count = 0;     // ring of chunks in flight: oldest at head
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_len = 8;
  int grid = 0;
  BatchArgs args;
  struct Slot {
    bool used = false, done = false;
    int64_t ticket = 0;
    int gen = 0;
    naj_system* sys = nullptr;
    int nrhs = 0;
    size_t tile0 = 0;
    double* xb = nullptr;
    float* fb = nullptr;
    double* b = nullptr;
    double* part = nullptr;
    double* x = nullptr;       // caller's answer array
  };
  std::vector<Slot> slots;
  std::unordered_map<int64_t, int> tickets;
  std::vector<int64_t> ready;  // found finished, not yet handed out by step
  int64_t next_ticket = 1;
};

namespace {

void server_release_slot(naj_server* sv, int i) {
  naj_server::Slot& sl = sv->slots[i];
  if (sl.sys) free_system(sl.sys);
  sv->pool.release(sl.xb);
  sv->pool.release(sl.fb);
  sv->pool.release(sl.b);
  sv->pool.release(sl.part);
  if (sl.used) sv->items.release(sl.tile0);
  if (sl.ticket) sv->tickets.erase(sl.ticket);
  sl = naj_server::Slot{};
}

void free_server(naj_server* sv) {
  if (!sv) return;
  for (int i = 0; i < (int)sv->slots.size(); ++i)
    if (sv->slots[i].used) server_release_slot(sv, i);
  if (sv->exec) (void)hipGraphExecDestroy(sv->exec);
  if (sv->graph) (void)hipGraphDestroy(sv->graph);
  for (void* p : {(void*)sv->d_sys, (void*)sv->d_ctrl, (void*)sv->d_vt, (void*)sv->d_tiles, (void*)sv->d_active,
                  (void*)sv->d_nactive, (void*)sv->d_sact, (void*)sv->d_nsact, (void*)sv->d_done,
                  (void*)sv->d_slot_done, (void*)sv->pool.base})
    if (p) (void)hipFree(p);
  if (sv->h_flags) (void)hipHostFree(sv->h_flags);
  if (sv->h_ctrl) (void)hipHostFree(sv->h_ctrl);
  for (auto& e : sv->evc)
    if (e) (void)hipEventDestroy(e);
  if (sv->ev_adm) (void)hipEventDestroy(sv->ev_adm);
  if (sv->adm) (void)hipStreamDestroy(sv->adm);
  delete sv;
}

// Reads the flags of a finished chunk: requests whose tag is set are done.
void server_scan(naj_server* sv, int buf) {
  const int* f = sv->h_flags + (size_t)buf * sv->max_slots;
  for (int i = 0; i < sv->max_slots; ++i) {
    naj_server::Slot& sl = sv->slots[i];
    if (sl.used && !sl.done && f[i] == sl.gen) {
      sl.done = true;
      sv->ready.push_back(sl.ticket);
    }
  }
}

// Retires the oldest chunk in flight (waiting for it when `block`): its flags are read.
// Returns false when there is none, or it has not finished and block is false.
bool server_retire(naj_server* sv, bool block, naj_status* rc) {
  *rc = NAJ_OK;
  if (sv->count == 0) return false;
  const int b = sv->head;
  hipError_t e = block ? hipEventSynchronize(sv->evc[b]) : hipEventQuery(sv->evc[b]);
  if (e == hipErrorNotReady) return false;
  if (e != hipSuccess) {
    *rc = fail(NAJ_EDEVICE, "chunk event: %s", hipGetErrorString(e));
    return false;
  }
  server_scan(sv, b);
  sv->head = (sv->head + 1) % naj_server::kRing;
  sv->count -= 1;
  return true;
}

}  // namespace

extern "C" {

naj_status naj_server_create(int64_t mem_budget, int32_t max_slots, int32_t max_rhs, const naj_opts* opts,
                             void* stream, naj_server** out) {
  g_err.clear();
  (void)hipGetLastError();
  if (!out) return fail(NAJ_EINVAL, "out is NULL");
  *out = nullptr;
  if (mem_budget < (1 << 20)) return fail(NAJ_EINVAL, "mem_budget must be at least 1 MiB");
  if (max_slots < 1 || max_slots > 65536) return fail(NAJ_EINVAL, "max_slots must be in [1, 65536]");
  if (max_rhs < 1 || max_rhs > kMaxRhs) return fail(NAJ_EINVAL, "max_rhs must be in [1, %d]", kMaxRhs);
  naj_opts o;
  if (opts) o = *opts;
  else naj_opts_default(&o);
  if (!(o.tol > 0.0) || o.max_iter < 1 || o.k0 < 2 || o.confirm_gap < 1 ||
      (o.precision != NAJ_FP64 && o.precision != NAJ_MIXED) || !(o.inner_tol > 0.0 && o.inner_tol < 1.0) ||
      o.max_refine < 1 || o.inner_stall < 1 || o.stop != NAJ_STOP_RELRES)
    return fail(NAJ_EINVAL, "invalid options (servers stop on the relative residual)");
  naj_server* sv = new naj_server();
  sv->opts = o;
  sv->max_slots = max_slots;
  sv->st = (hipStream_t)stream;
  sv->slots.assign(max_slots, naj_server::Slot{});
  naj_status rc = NAJ_OK;
#define SV_TRY(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      rc = fail(e_ == hipErrorOutOfMemory ? NAJ_ENOMEM : NAJ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
      free_server(sv);                                                                            \
      return rc;                                                                                  \
    }                                                                                             \
  } while (0)
  SV_TRY(hipGetDevice(&sv->device));
  SV_TRY(sv->pool.init((size_t)mem_budget));
  // work items: at most one per 64-row slice or 4 long rows, at 8 bytes of budget per row at least
  sv->tile_cap = (int)std::min<int64_t>(1 << 26, mem_budget / (64 * 8) + max_slots);
  sv->items.reset((size_t)sv->tile_cap);
  SV_TRY(hipMalloc((void**)&sv->d_sys, sizeof(BatchSys) * max_slots));
  SV_TRY(hipMalloc((void**)&sv->d_ctrl, sizeof(Ctrl) * max_slots * kMaxRhs));
  SV_TRY(hipMalloc((void**)&sv->d_vt, sizeof(PassView) * max_slots * kMaxRhs));
  SV_TRY(hipMalloc((void**)&sv->d_tiles, sizeof(BatchTile) * sv->tile_cap));
  SV_TRY(hipMalloc((void**)&sv->d_active, sizeof(int) * sv->tile_cap));
  SV_TRY(hipMalloc((void**)&sv->d_nactive, sizeof(int) * 64));
  SV_TRY(hipMalloc((void**)&sv->d_sact, sizeof(int) * max_slots));
  SV_TRY(hipMalloc((void**)&sv->d_nsact, sizeof(int) * 64));
  SV_TRY(hipMalloc((void**)&sv->d_done, sizeof(unsigned int) * 64));
  SV_TRY(hipMalloc((void**)&sv->d_slot_done, sizeof(int) * max_slots));
  SV_TRY(hipMemsetAsync(sv->d_sys, 0, sizeof(BatchSys) * max_slots, sv->st));   // nrhs 0: empty slots
  SV_TRY(hipMemsetAsync(sv->d_slot_done, 0, sizeof(int) * max_slots, sv->st));
  SV_TRY(hipMemsetAsync(sv->d_nactive, 0, sizeof(int) * 64, sv->st));
  SV_TRY(hipMemsetAsync(sv->d_nsact, 0, sizeof(int) * 64, sv->st));
  SV_TRY(hipHostMalloc((void**)&sv->h_flags, sizeof(int) * naj_server::kRing * max_slots, hipHostMallocDefault));
  SV_TRY(hipHostMalloc((void**)&sv->h_ctrl, sizeof(Ctrl) * kMaxRhs, hipHostMallocDefault));
  for (int q = 0; q < naj_server::kRing; ++q) SV_TRY(hipEventCreateWithFlags(&sv->evc[q], hipEventDisableTiming));
  SV_TRY(hipEventCreateWithFlags(&sv->ev_adm, hipEventDisableTiming));
  SV_TRY(hipStreamCreateWithFlags(&sv->adm, hipStreamNonBlocking));
  const bool mixed = o.precision == NAJ_MIXED;
  int occ = 0;
  int kpmax = 1;
  while (kpmax < max_rhs) kpmax <<= 1;
  sv->max_rhs = max_rhs;
  const void* pass_fn = batch_pass_kernel(mixed, kpmax);
  SV_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pass_fn, kBatchBlock, 0));
  hipDeviceProp_t prop;
  SV_TRY(hipGetDeviceProperties(&prop, sv->device));
  const int cus = prop.multiProcessorCount;
  sv->grid = std::max(1, std::max(1, occ) * cus);
  BatchArgs& A = sv->args;
  A.tiles = sv->d_tiles;
  A.sys = sv->d_sys;
  A.nsys = max_slots;
  A.active = sv->d_active;
  A.nactive = sv->d_nactive;
  A.sact = sv->d_sact;
  A.nsact = sv->d_nsact;
  A.done = sv->d_done;
  A.slot_done = sv->d_slot_done;
  A.nxcd = std::max(1, std::min(kMaxDomains, env_int("NAJ_NXCD", (cus % 8 == 0) ? 8 : 1)));
  A.tol = o.tol;
  A.inner_tol = o.inner_tol;
  A.max_iter = o.max_iter;
  A.restart = o.restart ? 1 : 0;
  A.confirm_gap = o.confirm_gap;
  A.k0 = o.k0;
  A.precision = mixed ? 1 : 0;
  A.max_refine = o.max_refine;
  A.inner_stall = o.inner_stall;
  sv->graph_len = std::max(1, env_int("NAJ_SERVER_CHUNK", 8));
  hipStream_t cap = nullptr;
  SV_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t ce = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (ce == hipSuccess) {
    hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(kCompactBlock), 0, cap, A);
    for (int q = 0; q < sv->graph_len; ++q) {
      void* kargs[] = {&A};
      if (ce == hipSuccess) ce = hipLaunchKernel(pass_fn, dim3(sv->grid), dim3(kBatchBlock), kargs, 0, cap);
      hipLaunchKernelGGL(k_batch_decide, dim3(max_slots), dim3(kDecideBlock), 0, cap, A);
    }
    ce = hipStreamEndCapture(cap, &sv->graph);
  }
  if (ce == hipSuccess) ce = hipGraphInstantiate(&sv->exec, sv->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  SV_TRY(ce);
  SV_TRY(hipStreamSynchronize(sv->st));
#undef SV_TRY
  *out = sv;
  return NAJ_OK;
}

naj_status naj_server_admit(naj_server* sv, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                            const double* vals, const double* D, int32_t nrhs, const double* b, const double* x0,
                            double tol, double* x, int64_t* ticket) {
  g_err.clear();
  (void)hipGetLastError();
  if (!sv || !ticket || !b || !x) return fail(NAJ_EINVAL, "server, b, x and ticket are required");
  if (nrhs < 1 || nrhs > sv->max_rhs) return fail(NAJ_EINVAL, "nrhs must be in [1, %d] (the server's max_rhs)", sv->max_rhs);
  if (n < 1) return fail(NAJ_EINVAL, "n must be >= 1");
  if (!(tol > 0.0)) tol = sv->opts.tol;
  const bool mixed = sv->opts.precision == NAJ_MIXED;
  int lk = 0;
  while ((1 << lk) < nrhs) ++lk;
  const size_t nv = (size_t)n << lk;
  if (nv * sizeof(double) * 4 >= (1ull << 32))
    return fail(NAJ_EINVAL, "n x right-hand sides too large for the server (solve it alone)");
  // a lower bound of what the request needs (matrix, vectors and, for a sorted layout, its row
  // permutation); beyond the whole budget it can never fit.  A sorted layout also takes temporaries
  // while it is built (about 12 bytes per nonzero and 20 per row); they are released on every exit
  // of the build, so a build that runs out of budget returns all of it and may be retried.
  const size_t vec_bytes = nv * (sizeof(double) * 4 + (mixed ? sizeof(float) * 5 : 0));
  const size_t need = (size_t)nnz * (sizeof(int32_t) + sizeof(double) + sizeof(float)) + vec_bytes;
  if (need > sv->pool.size()) return fail(NAJ_ENOMEM, "request needs about %zu bytes, budget is %zu", need, sv->pool.size());
  int slot = -1;
  for (int i = 0; i < sv->max_slots; ++i)
    if (!sv->slots[i].used) {
      slot = i;
      break;
    }
  if (slot < 0) return fail(NAJ_EBUSY, "no free slot");
  if (need > sv->pool.largest_free()) return fail(NAJ_EBUSY, "not enough free budget now");
  HIP_TRY(hipSetDevice(sv->device));
  naj_server::Slot& sl = sv->slots[slot];
  naj_system* s = nullptr;
  bool idle = true;   // no other request holds budget
  for (const naj_server::Slot& q : sv->slots) idle = idle && !q.used;
  naj_status rc = create_system_impl(n, nnz, rowptr, colidx, vals, D, sv->adm, &sv->pool, true, &s);
  if (rc == NAJ_ENOMEM && idle)
    return fail(NAJ_ENOMEM, "request does not fit the budget even with no other request admitted");
  if (rc == NAJ_ENOMEM) return fail(NAJ_EBUSY, "not enough free budget now (system)");
  if (rc != NAJ_OK) return rc;
  sl.sys = s;
  const int T = tile_slices_for(s, nrhs, sv->opts.precision);
  const int nlt = (int)((s->n_long + 3) / 4);
  const int ntiles = std::max(1, nlt + (int)((s->nslices + T - 1) / T));
  size_t tile0 = 0;
  if (!sv->items.alloc((size_t)ntiles, &tile0)) {
    free_system(s);
    sl = naj_server::Slot{};
    return fail(NAJ_EBUSY, "work-item table full");
  }
  sl.used = true;
  sl.tile0 = tile0;
  const int ym = nrhs > 1 ? 1 : s->ymode;   // as in batches
  sl.xb = (double*)sv->pool.alloc(nv * sizeof(double) * (mixed ? 2 : 3 + ym));
  sl.fb = mixed ? (float*)sv->pool.alloc(nv * sizeof(float) * 5) : nullptr;
  sl.b = (double*)sv->pool.alloc(nv * sizeof(double));
  sl.part = (double*)sv->pool.alloc(sizeof(double) * kPartStride * ntiles * nrhs);
  if (!sl.xb || (mixed && !sl.fb) || !sl.b || !sl.part) {
    server_release_slot(sv, slot);
    return fail(NAJ_EBUSY, "not enough free budget now (vectors)");
  }
  // right-hand sides and starting points into the interleaved buffers (admission stream)
  const int kp = 1 << lk;
  const dim3 g1(blocks_for((int64_t)nv, kAux * 4)), b1(kAux);
  hipLaunchKernelGGL(k_batch_load, g1, b1, 0, sv->adm, b, nrhs, kp, s->perm, s->n, sl.b);
  hipLaunchKernelGGL(k_batch_load, g1, b1, 0, sv->adm, x0, nrhs, kp, s->perm, s->n, sl.xb);
  HIP_TRY(hipGetLastError());
  // the caller's b and x0 may be freed or reused once this call returns: the copies finish first
  HIP_TRY(hipStreamSynchronize(sv->adm));
  BatchSys rec = {};
  rec.A = sell_of(s);
  rec.A.dom_bounds = nullptr;
  rec.dinv = s->dinv;
  rec.xb = sl.xb;
  rec.fb = sl.fb;
  rec.xs = (uint32_t)(nv * sizeof(double));
  rec.fs = (uint32_t)(nv * sizeof(float));
  rec.b = sl.b;
  rec.part = sl.part;
  rec.ctrl = sv->d_ctrl + (size_t)slot * kMaxRhs;
  rec.vt = sv->d_vt + (size_t)slot * kMaxRhs;
  rec.tol = tol;
  rec.lk = lk;
  rec.nrhs = nrhs;
  rec.tile0 = (int)tile0;
  rec.ntiles = ntiles;
  rec.ymode = ym;
  sl.gen = (int)(sv->next_ticket & 0x3fffffff) + 1;
  rec.gen = sl.gen;
  // the pass stream takes the slot after the admission work, between chunks
  HIP_TRY(hipEventRecord(sv->ev_adm, sv->adm));
  HIP_TRY(hipStreamWaitEvent(sv->st, sv->ev_adm, 0));
  const int work = std::max(ntiles, kMaxRhs);
  hipLaunchKernelGGL(k_server_admit, dim3((work + 255) / 256), dim3(256), 0, sv->st, sv->args, slot, rec, T, nlt);
  HIP_TRY(hipGetLastError());
  sl.nrhs = nrhs;
  sl.x = x;
  sl.done = false;
  sl.ticket = sv->next_ticket++;
  sv->tickets[sl.ticket] = slot;
  *ticket = sl.ticket;
  return NAJ_OK;
}

naj_status naj_server_step(naj_server* sv, int32_t chunks, int64_t* done, int32_t cap, int32_t* ndone) {
  g_err.clear();
  (void)hipGetLastError();
  if (!sv || (cap > 0 && !done) || !ndone) return fail(NAJ_EINVAL, "server and ndone are required");
  *ndone = 0;
  HIP_TRY(hipSetDevice(sv->device));
  naj_status rc = NAJ_OK;
  bool active = false;
  for (const auto& sl : sv->slots) active = active || (sl.used && !sl.done);
  if (!active || chunks <= 0) {
    while (server_retire(sv, true, &rc)) {   // nothing to run: collect every chunk in flight
    }
    if (rc != NAJ_OK) return rc;
  } else {
    for (int c = 0; c < chunks; ++c) {
      if (sv->count == naj_server::kRing) {   // ring full: wait for the oldest chunk
        server_retire(sv, true, &rc);
        if (rc != NAJ_OK) return rc;
      }
      const int b = (sv->head + sv->count) % naj_server::kRing;
      HIP_TRY(hipGraphLaunch(sv->exec, sv->st));
      HIP_TRY(hipMemcpyAsync(sv->h_flags + (size_t)b * sv->max_slots, sv->d_slot_done, sizeof(int) * sv->max_slots,
                             hipMemcpyDeviceToHost, sv->st));
      HIP_TRY(hipEventRecord(sv->evc[b], sv->st));
      sv->count += 1;
    }
    while (server_retire(sv, false, &rc)) {   // every chunk that has already finished
    }
    if (rc != NAJ_OK) return rc;
  }
  int k = 0;
  while (k < cap && !sv->ready.empty()) {
    done[k++] = sv->ready.front();
    sv->ready.erase(sv->ready.begin());
  }
  *ndone = k;
  return NAJ_OK;
}

naj_status naj_server_result(naj_server* sv, int64_t ticket, naj_result* res) {
  g_err.clear();
  (void)hipGetLastError();
  if (!sv || !res) return fail(NAJ_EINVAL, "server and res are required");
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(NAJ_EINVAL, "unknown ticket %lld", (long long)ticket);
  const int slot = it->second;
  naj_server::Slot& sl = sv->slots[slot];
  if (!sl.done) return fail(NAJ_EBUSY, "request %lld has not finished", (long long)ticket);
  HIP_TRY(hipSetDevice(sv->device));
  naj_system* s = sl.sys;
  // A request is found finished only after the chunk it finished in has completed, and no
  // later pass touches it, so its answer is read on the admission stream without waiting
  // for the chunks still in flight.  The slot leaves the table in pass-stream order.
  hipLaunchKernelGGL(k_batch_store, dim3(blocks_for(s->n * sl.nrhs, kAux * 4)), dim3(kAux), 0, sv->adm, sv->d_sys, slot,
                     sl.nrhs, s->perm, s->n, sl.x);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(sv->h_ctrl, sv->d_ctrl + (size_t)slot * kMaxRhs, sizeof(Ctrl) * sl.nrhs,
                         hipMemcpyDeviceToHost, sv->adm));
  hipLaunchKernelGGL(k_server_clear, dim3(1), dim3(64), 0, sv->st, sv->args, slot);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(sv->adm));
  const bool mixed = sv->opts.precision == NAJ_MIXED;
  naj_status worst = NAJ_OK;
  for (int j = 0; j < sl.nrhs; ++j) {
    const Ctrl& c = sv->h_ctrl[j];
    naj_result& r = res[j];
    r.status = c.status;
    r.iterations = mixed ? c.inner_total : c.iterations;
    r.restarts = mixed ? c.inner_restarts : c.restarts;
    r.confirmations = mixed ? c.outer : c.confirms;
    r.relres = c.relres;
    r.hist_len = 0;
    r.nrestart_log = 0;
    r.kernel_ms = 0.0;
    r.passes = c.passes;
    r.grid = sv->grid;
    if (c.status < 0 && (worst >= 0 || c.status < worst)) worst = (naj_status)c.status;
    if (worst >= 0 && c.status == ST_NOT_CONVERGED) worst = NAJ_NOT_CONVERGED;
  }
  server_release_slot(sv, slot);   // nothing reads the slot's memory any more
  if (worst == NAJ_EBREAKDOWN) return fail(NAJ_EBREAKDOWN, "NaN/Inf in a reduction of the request");
  return worst;
}

naj_status naj_server_info(const naj_server* sv, int64_t* bytes_used, int64_t* bytes_total, int32_t* slots_used,
                           int32_t* slots_total) {
  if (!sv) return fail(NAJ_EINVAL, "server is NULL");
  int used = 0;
  for (const auto& sl : sv->slots) used += sl.used ? 1 : 0;
  if (bytes_used) *bytes_used = (int64_t)sv->pool.in_use();
  if (bytes_total) *bytes_total = (int64_t)sv->pool.size();
  if (slots_used) *slots_used = used;
  if (slots_total) *slots_total = sv->max_slots;
  return NAJ_OK;
}

void naj_server_destroy(naj_server* sv) {
  if (!sv) return;
  (void)hipSetDevice(sv->device);
  (void)hipStreamSynchronize(sv->st);
  if (sv->adm) (void)hipStreamSynchronize(sv->adm);
  free_server(sv);
}

}  // extern "C"
