// Serving loop: continuous batching of encrypted GCN inferences on one GPU.
//
// The server owns n_slots execution slots, each with its own context (HIP
// stream at the default priority and scratch memory), worker thread and device
// arena, so up to n_slots requests run at once and their kernels overlap on the
// device.  A request names a plan (the graph's packing, node order, operands),
// the client's resident evaluation keys, the client's ciphertexts in host
// memory and a host destination for the result.
//
// Device memory is accounted in full: held = the resident evaluation key sets
// (each distinct set once, from its first request on) + per distinct plan its
// operands (the graph's masks and adjacency plaintexts, server-side data
// encoded once) and weight tables + every slot's arena + every slot's scratch.
// A request needs an arena of its inputs and every layer's outputs, and
// scratch for its batched launches (bounded from the plan: the key-switch chunk
// buffers, the rotated ciphertexts and inner sums, the encoder's chunk and a
// margin of ciphertext buffers); it is admitted to an idle slot when held,
// grown by what that slot's arena and scratch must grow, stays within the
// budget; idle slots' arenas and scratch are released first when that makes
// the difference.  An arena only grows, so in steady state a request allocates
// nothing (no hipMalloc / hipFree, which would synchronise the device across
// slots).  The first request of a plan encodes (or loads) its operands and
// builds its tables under the plan's lock; from then on any number of requests
// run the plan at once, reading it only.  The waiting queue is FIFO; a later
// request that fits may pass a head that does not, until the head has been
// passed 16 times (then the queue waits for it).  A slot's work for one
// request: upload the inputs, run every layer in the batched form, download
// the last layer's ciphertexts.  Latency = completion - submission on the
// server's steady clock.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
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
  size_t footprint = 0;     // arena bytes: inputs and layer outputs
  size_t scratch = 0;       // scratch bound of its batched launches
  double t_submit = 0, t_start = 0, t_done = 0;
  int status = 0;
  std::string err;
  bool done = false;
  int passed = 0;
};

struct Slot {
  ckks_ctx* c = nullptr;
  uint8_t* arena = nullptr;
  size_t cap = 0;           // arena bytes allocated
  size_t cap_pending = 0;   // arena bytes the admitted request needs (counted in held at admission)
  size_t scratch = 0;       // scratch bytes accounted (max of the bound admitted and the measured size)
  bool busy = false;
};

constexpr size_t ALIGN = 256;
size_t up(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

}  // namespace

struct ficgcn_server {
  std::vector<Slot> slots;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<uint64_t, Req> reqs;
  std::deque<uint64_t> waiting;
  std::set<const ckks_keys*> keys_seen;
  struct PlanState {
    std::mutex m;
    bool ready = false;
    const uint64_t* const* ops_host = nullptr;   // the first submitted request's operands_host
  };
  std::map<const ficgcn_plan*, std::unique_ptr<PlanState>> plans;
  size_t budget = 0, held = 0, peak = 0, resident = 0;
  uint64_t allocs = 0, overruns = 0;
  int running = 0, max_running = 0;
  uint64_t next_id = 1;
  bool stop = false;
  double t_first = -1, t_last = 0;
  ~ficgcn_server();
};

namespace ficgcn {

// the chunk budget of batched key switching (ks_batch.hip)
constexpr size_t KS_CHUNK = (size_t)3 << 30;

static size_t ct_bytes(const ckks_ctx* c, int level) { return (size_t)2 * (level + 1) * c->N * 8; }

// arena layout of one request: inputs, then each layer's outputs
static size_t request_arena(const ficgcn_plan* p, std::vector<size_t>* off = nullptr) {
  const ckks_ctx* c = p->ctx;
  size_t b = 0;
  auto take = [&](size_t n) {
    if (off) off->push_back(b);
    b += up(n);
  };
  take((size_t)p->layers[0].n_in_cts() * ct_bytes(c, p->layers[0].level_in));
  for (const LayerPlan& lp : p->layers) take((size_t)lp.n_packed() * ct_bytes(c, lp.level_in));
  return b;
}

// Scratch of the batched launches, by the buffers that grow with the plan (each kept by the
// slot's context at its largest size): the key-switch chunk buffers (sources and digits, jobs'
// accumulators and conversions; each pair at most one chunk budget plus one entry), per
// SpIntra-CA layer the rotated ciphertexts and inner sums of every packed ciphertext (one per
// rotation step) and the square's tensor products, the pre-activation outputs, the device
// encoder's chunk, and 64 ciphertexts at the widest level for everything else.
static size_t scratch_bound(const ficgcn_plan* p) {
  const ckks_ctx* c = p->ctx;
  const size_t N = c->N;
  size_t ks_src = 0, ks_job = 0, layers = 0, widest = 0;
  for (const LayerPlan& lp : p->layers) {
    const size_t l1 = lp.level_in + 1, ext = l1 + c->alpha, nd = (l1 + c->alpha - 1) / c->alpha;
    const size_t per_job = 2 * (ext + l1) * N * 8, per_src = (nd * ext + l1) * N * 8;
    const size_t np = (size_t)std::max(1, lp.n_packed()), ct = ct_bytes(c, lp.level_in);
    const size_t rots = layer_rotation_steps(lp).size();
    const size_t jobs = rots * np + (lp.act ? np : 0);
    ks_src = std::max(ks_src, std::min(jobs * per_src, KS_CHUNK) + per_src);
    ks_job = std::max(ks_job, std::min(jobs * per_job, KS_CHUNK) + per_job);
    layers += rots * np * ct + np * ct * 5 / 2;   // rotations / inner sums; tensor + pre-activation
    widest = std::max(widest, ct);
  }
  const size_t encoder = (size_t)32 * N * 40;
  return ks_src + ks_job + layers + encoder + 64 * widest;
}

// device bytes of a plan's weight tables (per-operation residues, fused-pass weights): at most
// 40 bytes per weight and limb, and 64 KiB of constants per layer
static size_t plan_tables(const ficgcn_plan* p) {
  size_t b = 0;
  for (const LayerPlan& lp : p->layers) b += (size_t)40 * lp.f_in * lp.f_out * (lp.level_in + 1) + (64 << 10);
  return b;
}

static size_t keys_bytes(const ckks_keys* k) {
  const ckks_ctx* c = k->ctx;
  const size_t nd = (size_t)(c->L + c->alpha - 1) / c->alpha;
  return k->swk.size() * nd * 2 * (size_t)(c->L + c->alpha) * c->N * 8 + (k->s_ntt ? (size_t)(c->L + c->alpha) * c->N * 8 : 0);
}

static size_t slot_scratch_now(const ckks_ctx* c) {
  size_t b = 0;
  for (const auto& s : c->scratch) b += s.second;
  return b;
}

// frees an idle slot's arena and scratch (its stream has no work left)
static void release_slot(ficgcn_server* s, Slot& sl) {
  if (sl.arena) (void)hipFree(sl.arena);
  sl.arena = nullptr;
  for (auto& b : sl.c->scratch) {
    if (b.first) (void)hipFree(b.first);
    b = {nullptr, 0};
  }
  s->held -= sl.cap + sl.scratch;
  sl.cap = sl.scratch = 0;
}

// pick the next admissible request for slot k (FIFO with bounded passing); caller holds the lock.
// Held memory after admission, by the first option that fits the budget: (a) as it is, the slot's
// arena and scratch grown to the request's; (b) the other idle slots released first; (c) also the
// slot's own arena and scratch released and taken anew at the request's size.
static bool pick(ficgcn_server* s, int k, uint64_t& id) {
  Slot& me = s->slots[k];
  for (size_t w = 0; w < s->waiting.size(); ++w) {
    Req& q = s->reqs[s->waiting[w]];
    const size_t mine = me.cap + me.scratch;
    const size_t others = s->held - s->resident - mine;
    size_t idle = 0;
    for (size_t o = 0; o < s->slots.size(); ++o)
      if ((int)o != k && !s->slots[o].busy) idle += s->slots[o].cap + s->slots[o].scratch;
    const size_t grown = std::max(me.cap, q.footprint) + std::max(me.scratch, q.scratch);
    const size_t fresh = q.footprint + q.scratch;
    int option = -1;
    if (s->resident + others + grown <= s->budget) option = 0;
    else if (s->resident + others - idle + grown <= s->budget) option = 1;
    else if (s->resident + others - idle + fresh <= s->budget) option = 2;
    if (option >= 0) {
      if (option >= 1)
        for (size_t o = 0; o < s->slots.size(); ++o)
          if ((int)o != k && !s->slots[o].busy && s->slots[o].cap + s->slots[o].scratch) release_slot(s, s->slots[o]);
      if (option == 2) release_slot(s, me);
      id = s->waiting[w];
      for (size_t m = 0; m < w; ++m) s->reqs[s->waiting[m]].passed += 1;
      s->waiting.erase(s->waiting.begin() + w);
      // the slot's share grows to what the request may use (the arena itself grows in run_request)
      const size_t grow_a = q.footprint > me.cap ? q.footprint - me.cap : 0;
      const size_t grow_s = q.scratch > me.scratch ? q.scratch - me.scratch : 0;
      s->held += grow_a + grow_s;
      me.scratch += grow_s;
      me.cap_pending = std::max(me.cap, q.footprint);
      s->peak = std::max(s->peak, s->held);
      return true;
    }
    if (q.passed >= 16) return false;   // the head has waited long enough
  }
  return false;
}

static void load_operands(ckks_ctx* c, ficgcn_plan* p, const uint64_t* const* host) {
  for (size_t li = 0; li < p->layers.size(); ++li) {
    const LayerPlan& lp = p->layers[li];
    const uint64_t* src = host[li];
    if (!src) FICGCN_THROW(EINVAL_, "missing host operands of a layer");
    for (size_t i = 0; i < lp.ops.size(); ++i) {
      ficgcn_status st = ficgcn_plan_load_operand(c, p, (uint32_t)li, i, src);
      if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
      src += (size_t)(lp.op_lv[i] + 1 + (lp.op_x[i] ? c->alpha : 0)) * c->N;
    }
  }
}

// the plan's operands and tables, once, by whichever of its requests runs first: loaded from the
// first submitted request's operands_host, or encoded
static void prepare(ficgcn_server* s, ckks_ctx* c, ficgcn_plan* p) {
  ficgcn_server::PlanState* ps;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    ps = s->plans.at(p).get();
  }
  std::lock_guard<std::mutex> lk(ps->m);
  if (ps->ready) return;
  if (ps->ops_host) {
    load_operands(c, p, ps->ops_host);
  } else {
    ficgcn_status st = ficgcn_plan_encode(c, p);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
  }
  prepare_plan_device(c, p);
  HIPCHECK(hipStreamSynchronize(c->stream));
  ps->ready = true;
}

static void run_request(ficgcn_server* s, Slot& sl, Req& q) {
  ckks_ctx* c = sl.c;
  ficgcn_plan* p = const_cast<ficgcn_plan*>(q.r.plan);
  const LayerPlan& l0 = p->layers[0];
  const LayerPlan& ll = p->layers.back();
  try {
    ensure_device(c);
    prepare(s, c, p);
    if (sl.cap_pending > sl.cap) {   // the arena grows (never shrinks while the slot works)
      if (sl.arena) {
        HIPCHECK(hipStreamSynchronize(c->stream));
        HIPCHECK(hipFree(sl.arena));
      }
      sl.arena = nullptr;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        sl.cap = sl.cap_pending;   // already counted in held at admission
        s->allocs += 1;
      }
      HIPCHECK(hipMalloc(&sl.arena, sl.cap));
    }
    std::vector<size_t> off;
    request_arena(p, &off);
    const size_t nl = p->layers.size();
    // inputs
    const size_t in_ct = ct_bytes(c, l0.level_in);
    uint8_t* din = sl.arena + off[0];
    if (q.r.seeded) {   // first polynomials from the client, the uniform parts rebuilt from their seed
      const size_t half = in_ct / 2;
      const uint8_t* src = (const uint8_t*)q.r.inputs_host;
      if (q.r.packed_bits) {
        // packed first polynomials land in each input's second half (rebuilt next), then unpack
        const int l1 = l0.level_in + 1;
        const size_t pk = (size_t)l1 * ((c->N * (size_t)q.r.packed_bits) >> 6) * 8;
        for (size_t i = 0; i < q.r.n_in; ++i)
          HIPCHECK(hipMemcpyAsync(din + i * in_ct + half, src + i * pk, pk, hipMemcpyHostToDevice, c->stream));
        pack_residues(c, (const uint64_t*)(din + half), in_ct / 8, (uint64_t*)din, in_ct / 8, l1, q.r.n_in,
                      (int)q.r.packed_bits, true);
      } else {
        for (size_t i = 0; i < q.r.n_in; ++i)
          HIPCHECK(hipMemcpyAsync(din + i * in_ct, src + i * half, half, hipMemcpyHostToDevice, c->stream));
      }
      expand_seeded(c, q.r.a_seed, q.r.a_id0, q.r.n_in, l0.level_in, (uint64_t*)din);
    } else {
      HIPCHECK(hipMemcpyAsync(din, q.r.inputs_host, q.r.n_in * in_ct, hipMemcpyHostToDevice, c->stream));
    }
    std::vector<const uint64_t*> cur(q.r.n_in);
    for (size_t i = 0; i < q.r.n_in; ++i) cur[i] = (const uint64_t*)(din + i * in_ct);
    for (size_t li = 0; li < nl; ++li) {
      const LayerPlan& lp = p->layers[li];
      const size_t oc = ct_bytes(c, lp.level_in);
      uint8_t* dout = sl.arena + off[1 + li];
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
}

static void worker(ficgcn_server* s, int k) {
  Slot& sl = s->slots[k];
  (void)hipSetDevice(sl.c->device);
  for (;;) {
    uint64_t id;
    Req* qp;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || pick(s, k, id); });
      if (s->stop) return;
      qp = &s->reqs[id];   // map nodes are stable
      sl.busy = true;
      s->running += 1;
      s->max_running = std::max(s->max_running, s->running);
      qp->t_start = now_ms();
    }
    run_request(s, sl, *qp);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      qp->t_done = now_ms();
      qp->done = true;
      // measured scratch: more than the bound admitted is counted (and reported as an overrun)
      const size_t now = slot_scratch_now(sl.c);
      if (now > sl.scratch) {
        s->overruns += 1;
        s->held += now - sl.scratch;
        sl.scratch = now;
        s->peak = std::max(s->peak, s->held);
      }
      sl.busy = false;
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
  for (Slot& sl : slots) {
    if (sl.c->stream) (void)hipStreamSynchronize(sl.c->stream);
    if (sl.arena) (void)hipFree(sl.arena);
    if (sl.c->stream) (void)hipStreamDestroy(sl.c->stream);
    sl.c->stream = nullptr;
    delete sl.c;
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
    Slot sl;
    sl.c = c;
    s->slots.push_back(sl);
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
  const ckks_ctx* sc = server->slots[0].c;
  if (pc->N != sc->N || pc->L != sc->L || pc->alpha != sc->alpha || pc->mod != sc->mod)
    FICGCN_THROW(EINVAL_, "the plan was built for other CKKS parameters");
  if ((int)req->n_in != p->layers[0].n_in_cts()) FICGCN_THROW(EPLAN_, "wrong number of input ciphertexts");
  if ((int)req->n_out != p->layers.back().n_packed()) FICGCN_THROW(EPLAN_, "wrong number of output ciphertexts");
  if (req->seeded && req->n_in > 0 && req->n_in - 1 > (size_t)(UINT32_MAX - req->a_id0))
    FICGCN_THROW(EINVAL_, "seeded input ids beyond 32 bits");
  if (req->packed_bits) {
    if (!req->seeded || req->packed_bits > 64) FICGCN_THROW(EINVAL_, "packed inputs must be seeded, at most 64 bits");
    for (int i = 0; i <= p->layers[0].level_in; ++i)
      if (req->packed_bits < 64 && (pc->mod[i] >> req->packed_bits)) FICGCN_THROW(EINVAL_, "packed width below a prime's bit length");
  }
  if (req->eval_keys->ctx && req->eval_keys->ctx->N != sc->N) FICGCN_THROW(EINVAL_, "keys of other parameters");
  Req q;
  q.r = *req;
  q.footprint = request_arena(p);
  q.scratch = scratch_bound(p);
  std::lock_guard<std::mutex> lk(server->mu);
  // resident memory this request brings: its key set, its plan's operands and tables, once each
  size_t add = 0;
  const bool new_keys = !server->keys_seen.count(req->eval_keys), new_plan = !server->plans.count(p);
  if (new_keys) add += keys_bytes(req->eval_keys);
  if (new_plan) add += plan_tables(p) + plan_operand_bytes(p);
  if (server->resident + add + q.footprint + q.scratch > server->budget)
    FICGCN_THROW(ENOMEM_, "request larger than the server's device budget (with resident keys and plans)");
  if (new_keys) server->keys_seen.insert(req->eval_keys);
  if (new_plan) {
    auto ps = std::unique_ptr<ficgcn_server::PlanState>(new ficgcn_server::PlanState());
    ps->ops_host = req->operands_host;
    server->plans.emplace(p, std::move(ps));
  }
  server->resident += add;
  server->held += add;
  server->peak = std::max(server->peak, server->held);
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
  out->footprint_bytes = q.footprint + q.scratch;
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
  out->resident_bytes = server->resident;
  out->arena_allocs = server->allocs;
  out->scratch_overruns = server->overruns;
  SV_END
}

}  // extern "C"
