// Serving loop: continuous batching of encrypted GCN inferences on one GPU.
//
// The server owns n_slots execution slots, each with its own context (HIP
// stream at the default priority and scratch memory) and worker thread, so
// up to n_slots requests run at once and their kernels overlap on the
// device.  A request names a plan (the graph's packing, node order,
// operands to encode), the client's resident evaluation keys, the client's
// ciphertexts in host memory and a host destination for the result.
// Admission is by device-memory footprint: a request's inputs, every
// layer's outputs and its encoded operands must fit under the budget next
// to the requests already running.  The waiting queue is FIFO; a later
// request that fits may pass a head that does not, until the head has been
// passed 16 times (then the queue waits for it).  A slot's life for one
// request: allocate, upload the inputs, encode the plan's operands, run
// every layer in the batched form, download the last layer's ciphertexts,
// free everything.  Latency = completion - submission on the server's
// steady clock.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "../../include/ficgcn.h"
#include "plan.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  ficgcn_request r{};
  size_t footprint = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  int status = 0;
  std::string err;
  bool done = false;
  int passed = 0;
};

}  // namespace

struct ficgcn_server {
  std::vector<ckks_ctx*> slots;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<uint64_t, Req> reqs;
  std::deque<uint64_t> waiting;
  size_t budget = 0, in_use = 0, peak = 0;
  int running = 0, max_running = 0;
  uint64_t next_id = 1;
  bool stop = false;
  double t_first = -1, t_last = 0;
  ~ficgcn_server();
};

namespace ficgcn {

static size_t ct_bytes(const ckks_ctx* c, int level) { return (size_t)2 * (level + 1) * c->N * 8; }

static size_t request_footprint(const ficgcn_plan* p) {
  const ckks_ctx* c = p->ctx;
  size_t b = plan_operand_bytes(p);
  const LayerPlan& l0 = p->layers[0];
  b += (size_t)l0.n_in_cts() * ct_bytes(c, l0.level_in);
  for (const LayerPlan& lp : p->layers) b += (size_t)lp.n_packed() * ct_bytes(c, lp.level_in);
  return b;
}

// pick the next admissible request (FIFO with bounded passing); caller holds the lock
static bool pick(ficgcn_server* s, uint64_t& id) {
  for (size_t k = 0; k < s->waiting.size(); ++k) {
    Req& q = s->reqs[s->waiting[k]];
    if (s->in_use + q.footprint <= s->budget) {
      id = s->waiting[k];
      for (size_t m = 0; m < k; ++m) s->reqs[s->waiting[m]].passed += 1;
      s->waiting.erase(s->waiting.begin() + k);
      return true;
    }
    if (q.passed >= 16) return false;   // the head has waited long enough
  }
  return false;
}

static void run_request(ckks_ctx* c, Req& q) {
  ficgcn_plan* p = const_cast<ficgcn_plan*>(q.r.plan);
  const LayerPlan& l0 = p->layers[0];
  const LayerPlan& ll = p->layers.back();
  std::vector<void*> blocks;
  try {
    ensure_device(c);
    // inputs
    const size_t in_ct = ct_bytes(c, l0.level_in);
    uint8_t* din = nullptr;
    HIPCHECK(hipMalloc(&din, std::max<size_t>(1, q.r.n_in * in_ct)));
    blocks.push_back(din);
    HIPCHECK(hipMemcpyAsync(din, q.r.inputs_host, q.r.n_in * in_ct, hipMemcpyHostToDevice, c->stream));
    // operands of this graph's plan
    ficgcn_status st = ficgcn_plan_encode(c, p);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    std::vector<const uint64_t*> cur(q.r.n_in);
    for (size_t i = 0; i < q.r.n_in; ++i) cur[i] = (const uint64_t*)(din + i * in_ct);
    for (size_t li = 0; li < p->layers.size(); ++li) {
      const LayerPlan& lp = p->layers[li];
      const size_t oc = ct_bytes(c, lp.level_in);
      uint8_t* dout = nullptr;
      HIPCHECK(hipMalloc(&dout, std::max<size_t>(1, lp.n_packed() * oc)));
      blocks.push_back(dout);
      std::vector<uint64_t*> outs(lp.n_packed());
      for (int i = 0; i < lp.n_packed(); ++i) outs[i] = (uint64_t*)(dout + i * oc);
      run_layer(c, q.r.eval_keys, p, (int)li, cur.data(), cur.size(), outs.data(), outs.size(), 1);
      cur.assign(outs.begin(), outs.end());
    }
    // the last layer's ciphertexts at its output level, back to the client
    const size_t words = (size_t)2 * (ll.level_out + 1) * c->N;
    for (size_t i = 0; i < cur.size(); ++i)
      HIPCHECK(hipMemcpyAsync(q.r.output_host + i * words, cur[i], words * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
  } catch (const Error& e) {
    q.status = e.code;
    q.err = e.msg;
  } catch (const std::exception& e) {
    q.status = EINVAL_;
    q.err = e.what();
  }
  (void)hipStreamSynchronize(c->stream);
  for (void* b : blocks) (void)hipFree(b);
  release_plan_device(p);
}

static void worker(ficgcn_server* s, int slot) {
  ckks_ctx* c = s->slots[slot];
  (void)hipSetDevice(c->device);
  for (;;) {
    uint64_t id;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || pick(s, id); });
      if (s->stop) return;
      Req& q = s->reqs[id];
      s->in_use += q.footprint;
      s->peak = std::max(s->peak, s->in_use);
      s->running += 1;
      s->max_running = std::max(s->max_running, s->running);
      q.t_start = now_ms();
    }
    Req* qp;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      qp = &s->reqs[id];   // map nodes are stable
    }
    run_request(c, *qp);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      qp->t_done = now_ms();
      qp->done = true;
      s->in_use -= qp->footprint;
      s->running -= 1;
      s->t_last = std::max(s->t_last, qp->t_done);
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace ficgcn

ficgcn_server::~ficgcn_server() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_work.notify_all();
  for (auto& t : workers)
    if (t.joinable()) t.join();
  for (ckks_ctx* c : slots) {
    if (c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
    delete c;
  }
}

using namespace ficgcn;

static ficgcn_status server_status(const Error& e) {
  set_error(e.msg);
  return (ficgcn_status)e.code;
}

#define SV_TRY try {
#define SV_END                                         \
  return FICGCN_OK;                                    \
  }                                                    \
  catch (const Error& e) { return server_status(e); }  \
  catch (const std::exception& e) {                    \
    set_error(e.what());                               \
    return FICGCN_EINVAL;                              \
  }

extern "C" {

ficgcn_status ficgcn_server_create(const ckks_params* params, uint32_t n_slots, uint64_t hbm_budget_bytes,
                                   ficgcn_server** out) {
  SV_TRY
  if (!params || !out || n_slots == 0 || n_slots > 16 || hbm_budget_bytes == 0) FICGCN_THROW(EINVAL_, "bad argument");
  std::unique_ptr<ficgcn_server> s(new ficgcn_server());
  s->budget = hbm_budget_bytes;
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  for (uint32_t k = 0; k < n_slots; ++k) {
    ckks_ctx* c = nullptr;
    ficgcn_status st = ckks_context_create(params, &c);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    s->slots.push_back(c);
    c->device = dev;
    HIPCHECK(hipStreamCreate(&c->stream));
  }
  for (uint32_t k = 0; k < n_slots; ++k) s->workers.emplace_back(worker, s.get(), (int)k);
  *out = s.release();
  SV_END
}

void ficgcn_server_destroy(ficgcn_server* server) { delete server; }

ficgcn_status ficgcn_server_submit(ficgcn_server* server, const ficgcn_request* req, uint64_t* id_out) {
  SV_TRY
  if (!server || !req || !id_out || !req->plan || !req->eval_keys || !req->inputs_host || !req->output_host)
    FICGCN_THROW(EINVAL_, "null argument");
  const ficgcn_plan* p = req->plan;
  const ckks_ctx* pc = p->ctx;
  const ckks_ctx* sc = server->slots[0];
  if (pc->N != sc->N || pc->L != sc->L || pc->alpha != sc->alpha || pc->mod != sc->mod)
    FICGCN_THROW(EINVAL_, "the plan was built for other CKKS parameters");
  if ((int)req->n_in != p->layers[0].n_in_cts()) FICGCN_THROW(EPLAN_, "wrong number of input ciphertexts");
  if ((int)req->n_out != p->layers.back().n_packed()) FICGCN_THROW(EPLAN_, "wrong number of output ciphertexts");
  Req q;
  q.r = *req;
  q.footprint = request_footprint(p);
  if (q.footprint > server->budget) FICGCN_THROW(ENOMEM_, "request larger than the server's device budget");
  std::lock_guard<std::mutex> lk(server->mu);
  for (const auto& kv : server->reqs)
    if (!kv.second.done && kv.second.r.plan == req->plan)
      FICGCN_THROW(EINVAL_, "a plan may serve one request at a time");
  q.t_submit = now_ms();
  if (server->t_first < 0) server->t_first = q.t_submit;
  const uint64_t id = server->next_id++;
  server->reqs.emplace(id, std::move(q));
  server->waiting.push_back(id);
  *id_out = id;
  server->cv_work.notify_all();
  SV_END
}

ficgcn_status ficgcn_server_wait(ficgcn_server* server, uint64_t id, ficgcn_request_result* out) {
  SV_TRY
  if (!server || !out) FICGCN_THROW(EINVAL_, "null argument");
  std::unique_lock<std::mutex> lk(server->mu);
  auto it = server->reqs.find(id);
  if (it == server->reqs.end()) FICGCN_THROW(EINVAL_, "unknown request");
  server->cv_done.wait(lk, [&] { return it->second.done; });
  const Req& q = it->second;
  out->status = q.status;
  out->queue_ms = q.t_start - q.t_submit;
  out->run_ms = q.t_done - q.t_start;
  out->latency_ms = q.t_done - q.t_submit;
  out->footprint_bytes = q.footprint;
  if (q.status != 0) {
    set_error(q.err);
    return (ficgcn_status)q.status;
  }
  SV_END
}

ficgcn_status ficgcn_server_stats(ficgcn_server* server, ficgcn_server_summary* out) {
  SV_TRY
  if (!server || !out) FICGCN_THROW(EINVAL_, "null argument");
  std::lock_guard<std::mutex> lk(server->mu);
  std::vector<double> lat;
  uint32_t failed = 0;
  for (const auto& kv : server->reqs)
    if (kv.second.done) {
      if (kv.second.status) ++failed;
      else lat.push_back(kv.second.t_done - kv.second.t_submit);
    }
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double f) {
    if (lat.empty()) return 0.0;
    // nearest rank
    size_t k = (size_t)std::ceil(f * lat.size());
    return lat[std::min(lat.size(), std::max<size_t>(1, k)) - 1];
  };
  std::memset(out, 0, sizeof(*out));
  out->completed = (uint32_t)lat.size();
  out->failed = failed;
  out->p50_ms = pct(0.50);
  out->p99_ms = pct(0.99);
  double sum = 0;
  for (double x : lat) sum += x;
  out->mean_ms = lat.empty() ? 0.0 : sum / lat.size();
  const double span = server->t_last - server->t_first;
  out->throughput_per_s = span > 0 ? lat.size() / (span * 1e-3) : 0.0;
  out->peak_bytes = server->peak;
  out->max_concurrent = (uint32_t)server->max_running;
  SV_END
}

}  // extern "C"
