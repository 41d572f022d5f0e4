// Serving core: continuous batching of curvature requests on one GPU.
//
// Requests (full H + OPG of a network, top-k eigenpairs of H, damped curvature
// queries against resident eigenpairs) enter a queue.  Worker slots, each with its own
// context and HIP stream, take the first queued request whose HBM footprint
// (workspace) fits in what is left of the caller's pool, so requests that arrive while
// others run are admitted as slots and memory free up and their work overlaps on the
// device.  With coalescing on, a slot that takes a damped query also takes every queued
// query against the same model and eigenpairs (up to a total batch size) and answers
// them with one call: every query is computed independently, so each result is the
// same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.h"

namespace {

using clock_t_ = std::chrono::steady_clock;

struct OwnedModel {  // deep copy of a hess_mlp's host arrays
  std::vector<int64_t> T;
  std::vector<int32_t> act;
  std::vector<const void*> W, b;
  hess_mlp view;
  void from(const hess_mlp& m) {
    T.assign(m.T, m.T + m.L);
    act.assign(m.act ? m.act : nullptr, m.act ? m.act + std::max(0, m.L - 2) : nullptr);
    W.assign(m.W, m.W + (m.L - 1));
    b.assign(m.b, m.b + (m.L - 1));
    view = m;
    view.T = T.data();
    view.act = act.empty() ? nullptr : act.data();
    view.W = W.data();
    view.b = b.data();
  }
};

struct Req {
  uint64_t id = 0;
  hess_request r;
  OwnedModel model;
  clock_t_::time_point t_submit, t_end;
  bool done = false;
  hess_status status = HESS_OK;
  size_t footprint = 0;
  int skipped = 0;
};

struct Block {
  size_t off, size;
};

}  // namespace

struct hess_server {
  int device = 0;
  char* pool = nullptr;
  size_t pool_bytes = 0;
  int coalesce = 1;
  int64_t max_batch = 4096;
  std::vector<Block> free_list;  // sorted by offset
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, Req*> reqs;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_id = 1;
  int64_t submitted = 0, completed = 0, failed = 0, batches = 0;
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

bool pool_alloc(hess_server* s, size_t bytes, size_t* off) {
  bytes = align_up(std::max<size_t>(bytes, 256));
  for (size_t i = 0; i < s->free_list.size(); ++i) {
    Block& b = s->free_list[i];
    if (b.size >= bytes) {
      *off = b.off;
      b.off += bytes;
      b.size -= bytes;
      if (b.size == 0) s->free_list.erase(s->free_list.begin() + i);
      return true;
    }
  }
  return false;
}

void pool_free(hess_server* s, size_t off, size_t bytes) {
  bytes = align_up(std::max<size_t>(bytes, 256));
  auto& fl = s->free_list;
  auto it = std::lower_bound(fl.begin(), fl.end(), off, [](const Block& b, size_t o) { return b.off < o; });
  it = fl.insert(it, Block{off, bytes});
  // merge with neighbours
  if (it + 1 != fl.end() && it->off + it->size == (it + 1)->off) {
    it->size += (it + 1)->size;
    fl.erase(it + 1);
  }
  if (it != fl.begin() && (it - 1)->off + (it - 1)->size == it->off) {
    (it - 1)->size += it->size;
    fl.erase(it);
  }
}

int64_t t1_of(const hess_mlp& m) { return m.T[0]; }
size_t dsize(int dtype) { return dtype == HESS_F64 ? 8 : 4; }

// Workspace of one request (or of a coalesced query batch of nq_total queries).
hess_status footprint(hess_ctx* ctx, const Req* q, int64_t nq_total, size_t* bytes) {
  const hess_request& r = q->r;
  size_t a = 0, b = 0;
  hess_status st;
  switch (r.kind) {
    case HESS_REQ_FULL:
      if ((st = hess_workspace_size(ctx, HESS_OP_EXACT, &q->model.view, &r.data, HESS_P_F32, 0, nullptr, &a)))
        return st;
      if ((st = hess_workspace_size(ctx, HESS_OP_OPG, &q->model.view, &r.data, HESS_P_F32, 0, nullptr, &b)))
        return st;
      *bytes = std::max(a, b);
      return HESS_OK;
    case HESS_REQ_TOPK: {
      hess_eig_opts o;
      std::memset(&o, 0, sizeof(o));
      o.which = 0;
      o.source = 0;
      o.prec = HESS_P_F32;
      o.oversample = 10;
      o.max_iter = 200;
      o.tol = r.tol;
      o.seed = r.seed;
      return hess_workspace_size(ctx, HESS_OP_TOPK, &q->model.view, &r.data, HESS_P_F32, r.K, &o, bytes);
    }
    case HESS_REQ_CURVATURE: {
      const int64_t K = r.K;
      return hess_workspace_size(ctx, HESS_OP_CURVATURE, nullptr, nullptr, 0, r.nq, &K, bytes);
    }
    case HESS_REQ_PREDVAR:
      if ((st = hess_workspace_size(ctx, HESS_OP_PREDVAR, &q->model.view, nullptr, 0, nq_total, nullptr, &a)))
        return st;
      // staging of the merged batch: inputs, classes, results
      *bytes = align_up(a) + align_up(nq_total * t1_of(q->model.view) * dsize(q->model.view.dtype)) +
               align_up(nq_total * 4) + align_up(nq_total * 8);
      return HESS_OK;
  }
  return HESS_E_ARG;
}

bool same_query_target(const Req* a, const Req* b) {
  const hess_request &x = a->r, &y = b->r;
  if (x.kind != HESS_REQ_PREDVAR || y.kind != HESS_REQ_PREDVAR) return false;
  if (x.fault_launch > 0 || y.fault_launch > 0) return false;
  if (x.K != y.K || x.lambda != y.lambda || x.Q != y.Q || x.delta != y.delta) return false;
  const hess_mlp &m = a->model.view, &n = b->model.view;
  if (m.L != n.L || m.dtype != n.dtype) return false;
  for (int k = 0; k < m.L; ++k)
    if (m.T[k] != n.T[k]) return false;
  for (int k = 0; k < m.L - 1; ++k)
    if (m.W[k] != n.W[k] || m.b[k] != n.b[k]) return false;
  for (int k = 0; k < m.L - 2; ++k)
    if (m.act[k] != n.act[k]) return false;
  return true;
}

hess_status run_full(hess_ctx* ctx, Req* q, void* ws, size_t wsb) {
  hess_status st = HESS_OK;
  if (q->r.H) st = hess_exact(ctx, &q->model.view, &q->r.data, HESS_P_F32, q->r.H, ws, wsb);
  if (st == HESS_OK && q->r.G) st = hess_opg(ctx, &q->model.view, &q->r.data, HESS_P_F32, q->r.G, ws, wsb);
  return st;
}

hess_status run_topk(hess_ctx* ctx, Req* q, void* ws, size_t wsb) {
  hess_eig_opts o;
  std::memset(&o, 0, sizeof(o));
  o.which = 0;
  o.source = 0;
  o.prec = HESS_P_F32;
  o.oversample = 10;
  o.max_iter = 200;
  o.tol = q->r.tol;
  o.seed = q->r.seed;
  hess_eig_info info;
  hess_status st = hess_topk_eig(ctx, &q->model.view, &q->r.data, q->r.K, &o, q->r.lambda, q->r.Q, &info, ws, wsb);
  return st == HESS_E_NOCONV ? HESS_OK : st;  // best iterate returned; accuracy is reported by the caller
}

// One damped-query call for a group of queries against the same target.
hess_status run_predvar_group(hess_ctx* ctx, hipStream_t stream, std::vector<Req*>& grp, char* ws, size_t wsb) {
  Req* q0 = grp[0];
  if (grp.size() == 1)
    return hess_predvar(ctx, &q0->model.view, q0->r.K, q0->r.lambda, q0->r.Q, q0->r.delta, q0->r.nq, q0->r.Xq,
                        q0->r.cls, q0->r.s, ws, wsb);
  int64_t nq = 0;
  bool any_cls = false;
  for (Req* q : grp) {
    nq += q->r.nq;
    any_cls = any_cls || q->r.cls != nullptr;
  }
  size_t pv = 0;
  hess_workspace_size(ctx, HESS_OP_PREDVAR, &q0->model.view, nullptr, 0, nq, nullptr, &pv);
  const size_t xs = dsize(q0->model.view.dtype) * t1_of(q0->model.view);
  char* X = ws + align_up(pv);
  int32_t* C = reinterpret_cast<int32_t*>(X + align_up(nq * xs));
  double* S = reinterpret_cast<double*>(reinterpret_cast<char*>(C) + align_up(nq * 4));
  int64_t o = 0;
  for (Req* q : grp) {
    hipMemcpyAsync(X + o * xs, q->r.Xq, q->r.nq * xs, hipMemcpyDeviceToDevice, stream);
    if (any_cls) {
      if (q->r.cls)
        hipMemcpyAsync(C + o, q->r.cls, q->r.nq * 4, hipMemcpyDeviceToDevice, stream);
      else
        hipMemsetAsync(C + o, 0xff, q->r.nq * 4, stream);  // -1 = arg-max class
    }
    o += q->r.nq;
  }
  hess_status st = hess_predvar(ctx, &q0->model.view, q0->r.K, q0->r.lambda, q0->r.Q, q0->r.delta, nq, X,
                                any_cls ? C : nullptr, S, ws, pv);
  if (st != HESS_OK) return st;
  o = 0;
  for (Req* q : grp) {
    hipMemcpyAsync(q->r.s, S + o, q->r.nq * 8, hipMemcpyDeviceToDevice, stream);
    o += q->r.nq;
  }
  return hipStreamSynchronize(stream) == hipSuccess ? HESS_OK : HESS_E_DEVICE;
}

void worker(hess_server* s, int slot) {
  (void)slot;
  hipSetDevice(s->device);
  hipStream_t stream = nullptr;
  hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
  hess_ctx* ctx = nullptr;
  hess_create(&ctx, s->device, stream);
  for (;;) {
    std::vector<Req*> grp;
    size_t off = 0, bytes = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop && s->queue.empty()) break;
        // first admissible request in arrival order; an old head request blocks others
        for (size_t i = 0; i < s->queue.size(); ++i) {
          Req* q = s->queue[i];
          if (pool_alloc(s, q->footprint, &off)) {
            bytes = q->footprint;
            grp.push_back(q);
            s->queue.erase(s->queue.begin() + i);
            break;
          }
          if (++q->skipped > 64 && i == 0) break;
        }
        if (!grp.empty()) break;
        s->cv_work.wait(lk);
      }
      if (grp.empty()) break;  // stopping
      if (s->coalesce && grp[0]->r.kind == HESS_REQ_PREDVAR) {
        // take every queued query against the same target while the batch and its memory fit
        int64_t nq = grp[0]->r.nq;
        size_t need = 0;
        for (size_t i = 0; i < s->queue.size();) {
          Req* q = s->queue[i];
          if (same_query_target(grp[0], q) && nq + q->r.nq <= s->max_batch) {
            footprint(ctx, grp[0], nq + q->r.nq, &need);
            size_t off2 = 0;
            pool_free(s, off, bytes);
            if (pool_alloc(s, need, &off2)) {
              off = off2;
              bytes = need;
              nq += q->r.nq;
              grp.push_back(q);
              s->queue.erase(s->queue.begin() + i);
              continue;
            }
            pool_alloc(s, bytes, &off);  // re-take the previous block (always fits: it was just freed)
          }
          ++i;
        }
        if (grp.size() > 1) s->batches++;
      }
    }
    hess_status st;
    char* ws = s->pool + off;
    const int32_t fault = grp[0]->r.fault_launch;
    if (fault > 0) hess_set_option(ctx, HESS_OPT_FAULT_AFTER, fault - 1);
    switch (grp[0]->r.kind) {
      case HESS_REQ_FULL: st = run_full(ctx, grp[0], ws, bytes); break;
      case HESS_REQ_TOPK: st = run_topk(ctx, grp[0], ws, bytes); break;
      case HESS_REQ_CURVATURE: {
        const hess_request& r = grp[0]->r;
        hs::Model mm;
        st = validate_mlp(nullptr, &grp[0]->model.view, mm, false);
        if (st == HESS_OK)
          st = hess_curvature(ctx, r.curv_mode, r.K, mm.P, r.lambda, r.Q, r.lam_tilde, r.nq,
                              static_cast<const double*>(r.Xq), r.s, ws, bytes);
        break;
      }
      default: st = run_predvar_group(ctx, stream, grp, ws, bytes); break;
    }
    if (fault > 0) hess_set_option(ctx, HESS_OPT_FAULT_AFTER, -1);
    const auto t_end = clock_t_::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      pool_free(s, off, bytes);
      for (Req* q : grp) {
        q->status = st;
        q->t_end = t_end;
        q->done = true;
        if (st == HESS_OK)
          s->completed++;
        else
          s->failed++;
      }
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  hess_destroy(ctx);
  hipStreamDestroy(stream);
}

}  // namespace

using namespace hs;

extern "C" {

hess_status hess_server_create(hess_server** out, int device, int n_slots, void* pool, size_t pool_bytes,
                               int coalesce) {
  if (!out || n_slots < 1 || n_slots > 64 || !pool || pool_bytes < 4096) return HESS_E_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HESS_E_DEVICE;
  hess_server* s = new hess_server();
  s->device = device;
  s->pool = static_cast<char*>(pool);
  s->pool_bytes = pool_bytes & ~size_t(255);
  s->coalesce = coalesce;
  s->free_list.push_back(Block{0, s->pool_bytes});
  for (int i = 0; i < n_slots; ++i) s->workers.emplace_back(worker, s, i);
  *out = s;
  return HESS_OK;
}

hess_status hess_server_submit(hess_server* s, const hess_request* r, uint64_t* id) {
  if (!s || !r || !id) return HESS_E_ARG;
  if (r->kind < HESS_REQ_FULL || r->kind > HESS_REQ_CURVATURE) return HESS_E_ARG;
  Model m;
  hess_status st = validate_mlp(nullptr, &r->model, m, true);
  if (st != HESS_OK) return st;
  if (r->kind == HESS_REQ_PREDVAR && (r->nq < 1 || !r->Xq || !r->s || !r->lambda || !r->Q)) return HESS_E_ARG;
  if (r->kind == HESS_REQ_CURVATURE &&
      (r->nq < 1 || r->K < 1 || r->K > m.P || !r->Xq || !r->s || !r->lambda || !r->Q || r->curv_mode < 0 ||
       r->curv_mode > HESS_CURV_FULL_INV))
    return HESS_E_ARG;
  if (r->kind != HESS_REQ_PREDVAR && r->kind != HESS_REQ_CURVATURE &&
      (st = validate_data(nullptr, &r->data, true)) != HESS_OK)
    return st;
  Req* q = new Req();
  q->r = *r;
  q->model.from(r->model);
  q->t_submit = clock_t_::now();
  hess_ctx* tmp = nullptr;  // workspace queries touch no device state
  st = footprint(tmp, q, r->kind == HESS_REQ_PREDVAR ? r->nq : 0, &q->footprint);
  if (st != HESS_OK) {
    delete q;
    return st;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (q->footprint > s->pool_bytes) {
    delete q;
    return HESS_E_BUDGET;
  }
  q->id = s->next_id++;
  s->reqs[q->id] = q;
  s->queue.push_back(q);
  s->submitted++;
  *id = q->id;
  s->cv_work.notify_one();
  return HESS_OK;
}

hess_status hess_server_wait(hess_server* s, uint64_t id, double* latency_ms) {
  if (!s) return HESS_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return HESS_E_ARG;
  Req* q = it->second;
  s->cv_done.wait(lk, [&] { return q->done; });
  if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(q->t_end - q->t_submit).count();
  const hess_status st = q->status;
  s->reqs.erase(it);
  delete q;
  return st;
}

hess_status hess_server_stats(hess_server* s, int64_t* out4) {
  if (!s || !out4) return HESS_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  out4[0] = s->submitted;
  out4[1] = s->completed;
  out4[2] = s->failed;
  out4[3] = s->batches;
  return HESS_OK;
}

hess_status hess_server_destroy(hess_server* s) {
  if (!s) return HESS_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return HESS_OK;
}

}  // extern "C"
