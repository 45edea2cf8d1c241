// extern "C" entry points: argument validation, then the device routines.
// No exception crosses the boundary; failures return a status and leave a
// thread-local message.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ficgcn.h"
#include "internal.h"
#include "ks_batch.h"

namespace ficgcn {
void decode_values(int N, const std::vector<double>& m, double scale, double* re, double* im, size_t n);
void crt_center(const std::vector<uint64_t>& mods, const uint64_t* res, int N, std::vector<double>& out);

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

template <typename F>
static ficgcn_status guard(F&& f) {
  try {
    f();
    return FICGCN_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return (ficgcn_status)e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return FICGCN_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return FICGCN_EINVAL;
  }
}

#define REQUIRE(cond, code, msg) \
  do {                           \
    if (!(cond)) FICGCN_THROW(code, msg); \
  } while (0)

static void check_level(const ckks_ctx* c, uint32_t level) {
  REQUIRE(c != nullptr, EINVAL_, "null context");
  REQUIRE((int)level < c->L, ELEVEL_, "level " + std::to_string(level) + " >= number of Q primes");
}

static void upload_ntt(ckks_ctx* c, const uint64_t* host, int n_limbs, uint64_t* dev, int n_polys,
                       int ext_level = -1) {
  const size_t bytes = (size_t)n_polys * n_limbs * c->N * 8;
  HIPCHECK(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c->stream));
  ntt_fwd(c, dev, n_limbs, ext_level >= 0 ? lm_ext(ext_level, c->L) : lm_q(n_limbs), n_polys, (size_t)n_limbs * c->N);
  HIPCHECK(hipStreamSynchronize(c->stream));   // host buffer may be released on return
}

void encode_batch_ext(ckks_ctx* c, const double* re, size_t count, size_t n, double scale, int level,
                      uint64_t* dev) {
  encode_gpu(c, re, nullptr, count, n, scale, level + 1 + c->alpha, lm_ext(level, c->L), dev);
}

void pt_load_ext(ckks_ctx* c, const uint64_t* host, int level, uint64_t* dev) {
  upload_ntt(c, host, level + 1 + c->alpha, dev, 1, level);
}

static const uint64_t* need_key(const ckks_keys* k, uint64_t tag) {
  REQUIRE(k != nullptr, EINVAL_, "null key set");
  auto it = k->swk.find(tag);
  REQUIRE(it != k->swk.end(), ENOKEY_, "missing switching key for tag " + std::to_string(tag));
  return it->second;
}

}  // namespace ficgcn

using namespace ficgcn;

// n rotations (cts[i] by steps[i] into outs[i]) as one key-switch batch:
// inputs given by the same pointer share one ModUp (hoisting)
static void rotate_batch(ckks_ctx* ctx, const ckks_keys* ek, const uint64_t* const* cts, uint32_t level,
                         const int64_t* steps, size_t n, uint64_t* const* outs) {
  const size_t N = ctx->N;
  const int l1 = level + 1;
  std::vector<const uint64_t*> srcs;
  std::map<const uint64_t*, int> src_of;
  std::vector<KSJob> jobs;
  std::vector<uint64_t*> gouts;
  std::vector<std::pair<uint64_t*, const uint64_t*>> copies;
  for (size_t i = 0; i < n; ++i) {
    REQUIRE(cts[i] && outs[i], EINVAL_, "null ciphertext");
    for (size_t j = 0; j < n; ++j)
      REQUIRE(outs[i] != cts[j] && (i == j || outs[i] != outs[j]), EINVAL_, "output buffers alias");
    const uint64_t g = galois_elt(ctx, steps[i]);
    if (g == 1) {
      copies.push_back({outs[i], cts[i]});
      continue;
    }
    const uint64_t* key = need_key(ek, g);
    auto it = src_of.find(cts[i]);
    if (it == src_of.end()) {
      it = src_of.emplace(cts[i], (int)srcs.size()).first;
      srcs.push_back(cts[i] + (size_t)l1 * N);
    }
    jobs.push_back(KSJob{key, cts[i], nullptr, nullptr, g, it->second, (int)gouts.size()});
    gouts.push_back(outs[i]);
  }
  for (auto& cp : copies) copy_d2d(ctx, cp.first, cp.second, (size_t)2 * l1 * N * 8);
  keyswitch_batch(ctx, (int)level, srcs, jobs, gouts, false);
}

extern "C" {

const char* ficgcn_last_error(void) { return g_err.c_str(); }

ficgcn_status ckks_context_create(const ckks_params* p, ckks_ctx** out) {
  return guard([&] {
    REQUIRE(p && out, EINVAL_, "null argument");
    REQUIRE(p->log_n >= 9 && p->log_n <= 17, EINVAL_, "log_n must be in [9, 17]");
    REQUIRE(p->n_q >= 1 && p->n_q <= 60 && p->n_p >= 1 && p->n_p <= 8, EINVAL_, "n_q in [1, 60], n_p in [1, 8]");
    std::unique_ptr<ckks_ctx> c(new ckks_ctx());
    c->log_n = (int)p->log_n;
    c->L = (int)p->n_q;
    c->alpha = (int)p->n_p;
    c->q_bits = (int)p->q_bits;
    c->p_bits = (int)p->p_bits;
    c->log_scale = (int)p->log_scale;
    build_context(c.get());
    *out = c.release();
  });
}

void ckks_ctx_destroy(ckks_ctx* ctx) { delete ctx; }

ficgcn_status ckks_ctx_set_stream(ckks_ctx* ctx, void* stream) {
  return guard([&] {
    REQUIRE(ctx, EINVAL_, "null context");
    ctx->stream = (hipStream_t)stream;
  });
}

ficgcn_status ckks_ctx_moduli(const ckks_ctx* ctx, uint64_t* out) {
  return guard([&] {
    REQUIRE(ctx && out, EINVAL_, "null argument");
    std::memcpy(out, ctx->mod.data(), ctx->mod.size() * 8);
  });
}

ficgcn_status ckks_galois_element(const ckks_ctx* ctx, int64_t step, uint64_t* g_out) {
  return guard([&] {
    REQUIRE(ctx && g_out, EINVAL_, "null argument");
    *g_out = galois_elt(const_cast<ckks_ctx*>(ctx), step);
  });
}

ficgcn_status ckks_sync(ckks_ctx* ctx) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    REQUIRE(ctx, EINVAL_, "null context");
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  });
}

// ---------------------------------------------------------------- keys
static uint64_t* alloc_swk(ckks_ctx* c) {
  uint64_t* p = nullptr;
  size_t bytes = (size_t)c->beta() * 2 * c->n_mod() * c->N * 8;
  if (hipMalloc(&p, bytes) != hipSuccess) FICGCN_THROW(ENOMEM_, "key allocation failed");
  return p;
}

ficgcn_status ckks_keygen(ckks_ctx* ctx, uint64_t seed, const int64_t* rot_steps, size_t n_steps, int with_relin,
                          ckks_keys** client_keys, ckks_keys** eval_keys) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    REQUIRE(ctx, EINVAL_, "null context");
    REQUIRE(n_steps == 0 || rot_steps, EINVAL_, "null rot_steps");
    const size_t N = ctx->N;
    const int nm = ctx->n_mod();
    std::unique_ptr<ckks_keys> cl(new ckks_keys()), ev(new ckks_keys());
    cl->ctx = ev->ctx = ctx;
    cl->has_secret = true;
    cl->seed = seed;
    HIPCHECK(hipMalloc(&cl->s_ntt, (size_t)nm * N * 8));
    sample_small_rns(ctx, cl->s_ntt, seed, 1, 0, 0, 0, nm, lm_q(nm));
    ntt_fwd(ctx, cl->s_ntt, nm, lm_q(nm), 1, 0);
    uint64_t* sp = (uint64_t*)ctx->buf(11, (size_t)nm * N * 8);
    auto make = [&](uint64_t tag) {
      if (ev->swk.count(tag)) return;
      if (tag == 0)
        ew_mul(ctx, sp, cl->s_ntt, cl->s_ntt, nm, lm_q(nm));
      else
        automorph_ntt(ctx, sp, cl->s_ntt, tag, nm, 1);
      uint64_t* k = alloc_swk(ctx);
      ev->swk[tag] = k;
      keygen_swk(ctx, seed, cl->s_ntt, sp, tag, k);
    };
    for (size_t i = 0; i < n_steps; ++i) {
      uint64_t g = galois_elt(ctx, rot_steps[i]);
      if (g != 1) make(g);
    }
    if (with_relin) make(0);
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    if (client_keys) *client_keys = cl.release();
    if (eval_keys) *eval_keys = ev.release();
  });
}

ficgcn_status ckks_keys_tags(const ckks_keys* keys, uint64_t* tags_out, size_t cap, size_t* n_out) {
  return guard([&] {
    REQUIRE(keys && n_out, EINVAL_, "null argument");
    *n_out = keys->swk.size();
    size_t i = 0;
    for (auto& kv : keys->swk) {
      if (tags_out && i < cap) tags_out[i] = kv.first;
      ++i;
    }
  });
}

ficgcn_status ckks_keys_export(ckks_ctx* ctx, const ckks_keys* keys, uint64_t tag, uint64_t* host_out) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    REQUIRE(ctx && host_out, EINVAL_, "null argument");
    const uint64_t* k = need_key(keys, tag);
    const size_t N = ctx->N;
    const int nm = ctx->n_mod();
    const size_t words = (size_t)ctx->beta() * 2 * nm * N;
    uint64_t* tmp = (uint64_t*)ctx->buf(12, words * 8);
    HIPCHECK(hipMemcpyAsync(tmp, k, words * 8, hipMemcpyDeviceToDevice, ctx->stream));
    ntt_inv(ctx, tmp, nm, lm_q(nm), ctx->beta() * 2, (size_t)nm * N);
    HIPCHECK(hipMemcpyAsync(host_out, tmp, words * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  });
}

ficgcn_status ckks_keys_import(ckks_ctx* ctx, ckks_keys* keys, uint64_t tag, const uint64_t* host_in) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    REQUIRE(ctx && keys && host_in, EINVAL_, "null argument");
    const size_t N = ctx->N;
    const int nm = ctx->n_mod();
    const size_t words = (size_t)ctx->beta() * 2 * nm * N;
    uint64_t* k;
    auto it = keys->swk.find(tag);
    if (it == keys->swk.end()) {
      k = alloc_swk(ctx);
      keys->swk[tag] = k;
    } else {
      k = it->second;
    }
    HIPCHECK(hipMemcpyAsync(k, host_in, words * 8, hipMemcpyHostToDevice, ctx->stream));
    ntt_fwd(ctx, k, nm, lm_q(nm), ctx->beta() * 2, (size_t)nm * N);
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  });
}

ficgcn_status ckks_keys_create_empty(ckks_ctx* ctx, ckks_keys** out) {
  return guard([&] {
    REQUIRE(ctx && out, EINVAL_, "null argument");
    ckks_keys* k = new ckks_keys();
    k->ctx = ctx;
    *out = k;
  });
}

void ckks_keys_destroy(ckks_keys* keys) { delete keys; }

// ---------------------------------------------------------------- encode / encrypt
ficgcn_status ckks_encode(ckks_ctx* ctx, const double* re, const double* im, size_t n, double scale, uint32_t level,
                          uint64_t* pt_dev) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(pt_dev && (re || n == 0), EINVAL_, "null argument");
    REQUIRE(n <= (size_t)ctx->N / 2, EINVAL_, "more values than slots");
    encode_gpu(ctx, re, im, 1, n, scale, (int)level + 1, lm_q((int)level + 1), pt_dev);
  });
}

ficgcn_status ckks_encode_batch(ckks_ctx* ctx, const double* re, size_t count, size_t n, double scale, uint32_t level,
                                uint64_t* pt_dev) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(pt_dev && re, EINVAL_, "null argument");
    REQUIRE(n <= (size_t)ctx->N / 2, EINVAL_, "more values than slots");
    encode_gpu(ctx, re, nullptr, count, n, scale, (int)level + 1, lm_q((int)level + 1), pt_dev);
  });
}

ficgcn_status ckks_pt_load(ckks_ctx* ctx, const uint64_t* host_coeffs, uint32_t level, uint64_t* pt_dev) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(host_coeffs && pt_dev, EINVAL_, "null argument");
    upload_ntt(ctx, host_coeffs, level + 1, pt_dev, 1);
  });
}

ficgcn_status ckks_encrypt(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* pt_dev, uint32_t level,
                           uint64_t seed, uint32_t ct_id, uint64_t* ct_dev) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(client_keys && client_keys->has_secret, EINVAL_, "encryption needs the client key set");
    REQUIRE(pt_dev && ct_dev, EINVAL_, "null argument");
    encrypt_sym(ctx, client_keys->s_ntt, pt_dev, level, seed, seed, ct_id, ct_dev);
  });
}

ficgcn_status ckks_encrypt_seeded(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* pt_dev, uint32_t level,
                                  uint64_t e_seed, uint64_t a_seed, uint32_t ct_id, uint64_t* ct_dev) {
  return guard([&] {
    check_level(ctx, level);
    REQUIRE(client_keys && client_keys->has_secret, EINVAL_, "encryption needs the client key set");
    REQUIRE(pt_dev && ct_dev, EINVAL_, "null argument");
    REQUIRE(a_seed != e_seed && a_seed != client_keys->seed, EINVAL_,
            "the public seed must differ from the error seed and the key generation seed");
    ensure_device(ctx);
    encrypt_sym(ctx, client_keys->s_ntt, pt_dev, level, e_seed, a_seed, ct_id, ct_dev);
  });
}

ficgcn_status ckks_expand_seeded(ckks_ctx* ctx, uint64_t a_seed, uint32_t ct_id0, size_t count, uint32_t level,
                                 uint64_t* cts_dev) {
  return guard([&] {
    check_level(ctx, level);
    if (count == 0) return;
    REQUIRE(cts_dev, EINVAL_, "null argument");
    REQUIRE(count - 1 <= (size_t)(UINT32_MAX - ct_id0), EINVAL_, "ciphertext ids beyond 32 bits");
    ensure_device(ctx);
    expand_seeded(ctx, a_seed, ct_id0, count, (int)level, cts_dev);
  });
}

ficgcn_status ckks_pack_residues(ckks_ctx* ctx, const uint64_t* in_dev, size_t n_limbs, uint32_t bits,
                                 uint64_t* out_dev) {
  return guard([&] {
    REQUIRE(ctx, EINVAL_, "null context");
    REQUIRE(bits >= 1 && bits <= 64, EINVAL_, "bits per residue must lie in 1..64");
    REQUIRE(n_limbs <= 65535, EINVAL_, "at most 65535 limbs per call");
    if (n_limbs == 0) return;
    REQUIRE(in_dev && out_dev, EINVAL_, "null argument");
    ensure_device(ctx);
    pack_residues(ctx, in_dev, 0, out_dev, 0, (int)n_limbs, 1, (int)bits, false);
  });
}

ficgcn_status ckks_unpack_residues(ckks_ctx* ctx, const uint64_t* in_dev, size_t n_limbs, uint32_t bits,
                                   uint64_t* out_dev) {
  return guard([&] {
    REQUIRE(ctx, EINVAL_, "null context");
    REQUIRE(bits >= 1 && bits <= 64, EINVAL_, "bits per residue must lie in 1..64");
    REQUIRE(n_limbs <= 65535, EINVAL_, "at most 65535 limbs per call");
    if (n_limbs == 0) return;
    REQUIRE(in_dev && out_dev, EINVAL_, "null argument");
    ensure_device(ctx);
    pack_residues(ctx, in_dev, 0, out_dev, 0, (int)n_limbs, 1, (int)bits, true);
  });
}

ficgcn_status ckks_decrypt(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* ct_dev, uint32_t level,
                           double scale, double* re, double* im, size_t n_slots) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(client_keys && client_keys->has_secret, EINVAL_, "decryption needs the client key set");
    REQUIRE(ct_dev && (re || im), EINVAL_, "null argument");
    const size_t N = ctx->N;
    const int l1 = level + 1;
    uint64_t* m = (uint64_t*)ctx->buf(13, (size_t)l1 * N * 8);
    decrypt_core(ctx, ct_dev, client_keys->s_ntt, level, m);
    ntt_inv(ctx, m, l1, lm_q(l1), 1, 0);
    std::vector<uint64_t> host((size_t)l1 * N);
    HIPCHECK(hipMemcpyAsync(host.data(), m, host.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    std::vector<uint64_t> mods(ctx->mod.begin(), ctx->mod.begin() + l1);
    std::vector<double> coef;
    crt_center(mods, host.data(), (int)N, coef);
    decode_values((int)N, coef, scale, re, im, n_slots);
  });
}

// ---------------------------------------------------------------- transfers
ficgcn_status ckks_ct_load(ckks_ctx* ctx, const uint64_t* host_coeffs, uint32_t level, uint64_t* ct_dev) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(host_coeffs && ct_dev, EINVAL_, "null argument");
    upload_ntt(ctx, host_coeffs, level + 1, ct_dev, 2);
  });
}

ficgcn_status ckks_poly_store(ckks_ctx* ctx, const uint64_t* dev, uint32_t level, uint32_t n_polys,
                              uint64_t* host_coeffs) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(dev && host_coeffs && n_polys >= 1, EINVAL_, "bad argument");
    const size_t N = ctx->N;
    const int l1 = level + 1;
    const size_t words = (size_t)n_polys * l1 * N;
    uint64_t* tmp = (uint64_t*)ctx->buf(14, words * 8);
    HIPCHECK(hipMemcpyAsync(tmp, dev, words * 8, hipMemcpyDeviceToDevice, ctx->stream));
    ntt_inv(ctx, tmp, l1, lm_q(l1), (int)n_polys, (size_t)l1 * N);
    HIPCHECK(hipMemcpyAsync(host_coeffs, tmp, words * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
  });
}

ficgcn_status ckks_ntt(ckks_ctx* ctx, uint64_t* dev, uint32_t n_limbs, uint32_t first_mod, int inverse) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    REQUIRE(ctx && dev, EINVAL_, "null argument");
    REQUIRE(first_mod + n_limbs <= (uint32_t)ctx->n_mod(), EINVAL_, "limb range outside the modulus chain");
    LimbMap map{(int)first_mod, 1 << 30, 0};
    if (inverse)
      ntt_inv(ctx, dev, (int)n_limbs, map, 1, 0);
    else
      ntt_fwd(ctx, dev, (int)n_limbs, map, 1, 0);
  });
}

// ---------------------------------------------------------------- evaluation
ficgcn_status ckks_rotate_hoisted(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* ct_dev, uint32_t level,
                                  const int64_t* steps, size_t k, uint64_t* const* outs) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(ct_dev && (k == 0 || (steps && outs)), EINVAL_, "null argument");
    std::vector<const uint64_t*> cts(k, ct_dev);
    rotate_batch(ctx, eval_keys, cts.data(), level, steps, k, outs);
  });
}

ficgcn_status ckks_rotate_batch(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* const* cts, uint32_t level,
                                const int64_t* steps, size_t n, uint64_t* const* outs) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(n == 0 || (cts && steps && outs), EINVAL_, "null argument");
    rotate_batch(ctx, eval_keys, cts, level, steps, n, outs);
  });
}

ficgcn_status ckks_pt_mul_acc(ckks_ctx* ctx, uint64_t* acc_dev, uint32_t level, const uint64_t* const* cts,
                              const uint64_t* const* pts, size_t k) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(acc_dev && (k == 0 || (cts && pts)), EINVAL_, "null argument");
    for (size_t b = 0; b < k; b += PtrList::MAX) {
      PtrList c{}, p{};
      int n = (int)std::min<size_t>(PtrList::MAX, k - b);
      for (int i = 0; i < n; ++i) {
        REQUIRE(cts[b + i] && pts[b + i], EINVAL_, "null operand");
        c.p[i] = cts[b + i];
        p.p[i] = pts[b + i];
      }
      pmul_acc(ctx, acc_dev, c, p, n, level + 1);
    }
  });
}

ficgcn_status ckks_scalar_mul_acc(ckks_ctx* ctx, uint64_t* acc_dev, uint32_t level, const uint64_t* const* cts,
                                  const int64_t* consts, size_t k) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(acc_dev && (k == 0 || (cts && consts)), EINVAL_, "null argument");
    const int l1 = level + 1;
    std::vector<uint64_t> host(k * l1 * 2);
    for (size_t t = 0; t < k; ++t)
      for (int i = 0; i < l1; ++i) {
        uint64_t q = ctx->mod[i];
        int64_t v = consts[t];
        uint64_t r = v >= 0 ? (uint64_t)v % q : (q - (uint64_t)(-(v + 1)) % q - 1) % q;
        host[(t * l1 + i) * 2] = r;
        host[(t * l1 + i) * 2 + 1] = shoup(r, q);
      }
    uint64_t* dev = (uint64_t*)ctx->buf(15, std::max<size_t>(8, host.size() * 8));
    HIPCHECK(hipMemcpyAsync(dev, host.data(), host.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    for (size_t b = 0; b < k; b += PtrList::MAX) {
      PtrList c{};
      int n = (int)std::min<size_t>(PtrList::MAX, k - b);
      for (int i = 0; i < n; ++i) {
        REQUIRE(cts[b + i], EINVAL_, "null operand");
        c.p[i] = cts[b + i];
      }
      smul_acc(ctx, acc_dev, c, dev + b * l1 * 2, n, l1);
    }
    HIPCHECK(hipStreamSynchronize(ctx->stream));   // host constants must outlive the copy
  });
}

ficgcn_status ckks_add(ckks_ctx* ctx, uint64_t* acc_dev, const uint64_t* in_dev, uint32_t level) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(acc_dev && in_dev, EINVAL_, "null argument");
    add_inplace(ctx, acc_dev, in_dev, level + 1, 2);
  });
}

ficgcn_status ckks_rescale(ckks_ctx* ctx, uint64_t* ct_dev, uint32_t level) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(ct_dev, EINVAL_, "null argument");
    REQUIRE(level >= 1, ELEVEL_, "rescale at level 0");
    rescale_inplace(ctx, ct_dev, (int)level);
  });
}

static bool ntt_split_ok(const ckks_ctx* c, int l1) {
  const int l2 = c->log_n - l1;
  return l1 >= 4 && l1 <= 9 && l2 >= 4 && l2 <= 9;
}

static bool ntt_cols_ok(int v) { return v == 1 || v == 2 || v == 4 || v == 8 || v == 16; }

ficgcn_status ckks_ntt_config(ckks_ctx* ctx, int32_t split, int32_t cols_column, int32_t cols_row) {
  return guard([&] {
    REQUIRE(ctx, EINVAL_, "null context");
    REQUIRE(split == 0 || ntt_split_ok(ctx, split), EINVAL_, "NTT split outside 2^4..2^9 points per pass");
    REQUIRE(ntt_cols_ok(cols_column) && ntt_cols_ok(cols_row), EINVAL_, "NTT widths must be 1, 2, 4, 8 or 16");
    ctx->ntt_split = split;
    ctx->ntt_cols[0] = cols_column;
    ctx->ntt_cols[1] = cols_row;
  });
}

ficgcn_status ckks_ntt_autotune(ckks_ctx* ctx, uint32_t n_limbs, int32_t* cols_out) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    REQUIRE(ctx && n_limbs >= 1 && n_limbs <= (uint32_t)ctx->n_mod(), EINVAL_, "bad argument");
    // a key-switch batch's shape: 16 polynomials of n_limbs limbs in one launch
    constexpr int NP = 16;
    const size_t words = (size_t)NP * n_limbs * ctx->N;
    const size_t ps = (size_t)n_limbs * ctx->N;
    uint64_t* d = (uint64_t*)ctx->buf(16, words * 8);
    // residues spread over [0, q): the transform's timing depends on the data
    for (int p = 0; p < NP; ++p) sample_uniform(ctx, d + p * ps, 0, 99, (uint32_t)p, 0, (int)n_limbs, lm_q((int)n_limbs), 0);
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    const bool prof = ctx->profiling;
    ctx->profiling = false;
    float best = 1e30f;
    int bc[3] = {ctx->ntt_cols[0], ctx->ntt_cols[1], ctx->ntt_split};
    const int mid = ctx->log_n / 2;
    for (int l1 : {mid - 1, mid, mid + 1}) {
      if (!ntt_split_ok(ctx, l1)) continue;
      for (int c0 : {4, 8, 16})
        for (int c1 : {2, 4, 8, 16}) {
          ctx->ntt_split = l1;
          ctx->ntt_cols[0] = c0;
          ctx->ntt_cols[1] = c1;
          ntt_fwd(ctx, d, (int)n_limbs, lm_q((int)n_limbs), NP, ps);   // warm-up
          ntt_inv(ctx, d, (int)n_limbs, lm_q((int)n_limbs), NP, ps);
          HIPCHECK(hipEventRecord(e0, ctx->stream));
          for (int r = 0; r < 5; ++r) {
            ntt_fwd(ctx, d, (int)n_limbs, lm_q((int)n_limbs), NP, ps);
            ntt_inv(ctx, d, (int)n_limbs, lm_q((int)n_limbs), NP, ps);
          }
          HIPCHECK(hipEventRecord(e1, ctx->stream));
          HIPCHECK(hipEventSynchronize(e1));
          float ms = 0;
          HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best) {
            best = ms;
            bc[0] = c0;
            bc[1] = c1;
            bc[2] = l1;
          }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profiling = prof;
    ctx->ntt_cols[0] = bc[0];
    ctx->ntt_cols[1] = bc[1];
    ctx->ntt_split = bc[2];
    if (cols_out) {
      cols_out[0] = bc[0];
      cols_out[1] = bc[1];
      cols_out[2] = bc[2];
    }
  });
}

ficgcn_status ficgcn_profile_enable(ckks_ctx* ctx, int on) {
  return guard([&] {
    REQUIRE(ctx, EINVAL_, "null context");
    ctx->profiling = on != 0;
  });
}

ficgcn_status ficgcn_profile_read(ckks_ctx* ctx, const char* kernel, double* ms_total, uint64_t* launches) {
  return guard([&] {
    REQUIRE(ctx && kernel && ms_total && launches, EINVAL_, "null argument");
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    double tot = 0;
    uint64_t n = 0;
    auto it = ctx->prof.find(kernel);
    if (it != ctx->prof.end()) {
      for (auto& ev : it->second) {
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, ev.first, ev.second));
        tot += ms;
        ++n;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
      }
      ctx->prof.erase(it);
    }
    *ms_total = tot;
    *launches = n;
  });
}

ficgcn_status ckks_mul_relin(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* x_dev, const uint64_t* y_dev,
                             uint32_t level, uint64_t* out_dev) {
  return guard([&] {
    if (ctx) ensure_device(ctx);
    check_level(ctx, level);
    REQUIRE(x_dev && y_dev && out_dev, EINVAL_, "null argument");
    REQUIRE(out_dev != x_dev && out_dev != y_dev, EINVAL_, "output aliases an input");
    const uint64_t* rk = need_key(eval_keys, 0);
    const size_t N = ctx->N;
    const int l1 = level + 1, ext = l1 + ctx->alpha;
    const int nd = (l1 + ctx->alpha - 1) / ctx->alpha;
    uint64_t* d = (uint64_t*)ctx->buf(22, (size_t)3 * l1 * N * 8);
    tensor(ctx, x_dev, y_dev, d, level);
    uint64_t* D = (uint64_t*)ctx->buf(20, (size_t)nd * ext * N * 8);
    uint64_t* acc = (uint64_t*)ctx->buf(21, (size_t)2 * ext * N * 8);
    modup(ctx, d + (size_t)2 * l1 * N, level, D);
    keymac(ctx, acc, D, rk, level, 1);
    moddown(ctx, acc, level, out_dev, d, 1, d + (size_t)l1 * N);
  });
}

}  // extern "C"

// ---------------------------------------------------------------- operands
// Level and scale checks of the descriptor forms; nothing touches the device
// before they pass.
static void check_op(const ckks_ctx* c, const ckks_operand* op, uint32_t n_poly, const char* what,
                     bool fresh_ok = false) {
  REQUIRE(c != nullptr, EINVAL_, "null context");
  REQUIRE(op != nullptr && op->data != nullptr, EINVAL_, std::string("null ") + what);
  REQUIRE(op->n_poly == n_poly, EINVAL_,
          std::string(what) + (n_poly == 2 ? " is not a ciphertext (n_poly != 2)" : " is not a plaintext (n_poly != 1)"));
  check_level(c, op->level);
  // an accumulator may be fresh (scale 0: it takes its first product's scale)
  REQUIRE((op->scale > 0.0 || (fresh_ok && op->scale == 0.0)) && std::isfinite(op->scale), ESCALE_,
          std::string(what) + ": scale must be positive");
}

static void same_level(const ckks_operand* a, const ckks_operand* b, const char* what) {
  REQUIRE(a->level == b->level, ELEVEL_,
          std::string(what) + ": level " + std::to_string(b->level) + " against " + std::to_string(a->level));
}

static bool scale_eq(double a, double b) { return std::fabs(a - b) <= 1e-9 * std::fabs(a); }

// acc's scale: 0 = fresh (takes the first product's), else every product must carry it
static double product_scale(const ckks_operand* acc, double first, const char* what) {
  if (acc->scale == 0.0) return first;
  REQUIRE(scale_eq(acc->scale, first), ESCALE_,
          std::string(what) + ": product scale " + std::to_string(first) + " against accumulator " +
              std::to_string(acc->scale));
  return acc->scale;
}

extern "C" {

ficgcn_status ckks_encrypt_op(ckks_ctx* ctx, const ckks_keys* client_keys, const ckks_operand* pt, uint64_t seed,
                              uint32_t ct_id, ckks_operand* ct) {
  return guard([&] {
    check_op(ctx, pt, 1, "plaintext");
    REQUIRE(ct && ct->data && ct->n_poly == 2, EINVAL_, "output is not a ciphertext buffer");
    const ficgcn_status st = ckks_encrypt(ctx, client_keys, pt->data, pt->level, seed, ct_id, ct->data);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    ct->level = pt->level;
    ct->scale = pt->scale;
  });
}

ficgcn_status ckks_decrypt_op(ckks_ctx* ctx, const ckks_keys* client_keys, const ckks_operand* ct, double* re,
                              double* im, size_t n_slots) {
  return guard([&] {
    check_op(ctx, ct, 2, "ciphertext");
    const ficgcn_status st = ckks_decrypt(ctx, client_keys, ct->data, ct->level, ct->scale, re, im, n_slots);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
  });
}

ficgcn_status ckks_rotate_hoisted_op(ckks_ctx* ctx, const ckks_keys* eval_keys, const ckks_operand* in,
                                     const int64_t* steps, size_t k, ckks_operand* outs) {
  return guard([&] {
    check_op(ctx, in, 2, "input ciphertext");
    REQUIRE(k == 0 || (steps && outs), EINVAL_, "null argument");
    std::vector<uint64_t*> o(k);
    for (size_t i = 0; i < k; ++i) {
      REQUIRE(outs[i].data && outs[i].n_poly == 2, EINVAL_, "output " + std::to_string(i) + " is not a ciphertext");
      REQUIRE(outs[i].level == in->level, ELEVEL_, "output " + std::to_string(i) + " is at another level");
      o[i] = outs[i].data;
    }
    const ficgcn_status st = ckks_rotate_hoisted(ctx, eval_keys, in->data, in->level, steps, k, o.data());
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    for (size_t i = 0; i < k; ++i) outs[i].scale = in->scale;
  });
}

ficgcn_status ckks_pt_mul_acc_op(ckks_ctx* ctx, ckks_operand* acc, const ckks_operand* cts, const ckks_operand* pts,
                                 size_t k) {
  return guard([&] {
    check_op(ctx, acc, 2, "accumulator", true);
    REQUIRE(k == 0 || (cts && pts), EINVAL_, "null argument");
    double sc = acc->scale;
    std::vector<const uint64_t*> c(k), p(k);
    for (size_t i = 0; i < k; ++i) {
      check_op(ctx, &cts[i], 2, "ciphertext");
      check_op(ctx, &pts[i], 1, "plaintext");
      same_level(acc, &cts[i], "ciphertext");
      same_level(acc, &pts[i], "plaintext");
      const ckks_operand cur{acc->data, acc->level, 2, sc};
      sc = product_scale(&cur, cts[i].scale * pts[i].scale, "pt_mul_acc");
      c[i] = cts[i].data;
      p[i] = pts[i].data;
    }
    const ficgcn_status st = ckks_pt_mul_acc(ctx, acc->data, acc->level, c.data(), p.data(), k);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    acc->scale = sc;
  });
}

ficgcn_status ckks_scalar_mul_acc_op(ckks_ctx* ctx, ckks_operand* acc, const ckks_operand* cts, const int64_t* consts,
                                     double const_scale, size_t k) {
  return guard([&] {
    check_op(ctx, acc, 2, "accumulator", true);
    REQUIRE(k == 0 || (cts && consts), EINVAL_, "null argument");
    REQUIRE(const_scale > 0.0 && std::isfinite(const_scale), ESCALE_, "constant scale must be positive");
    double sc = acc->scale;
    std::vector<const uint64_t*> c(k);
    for (size_t i = 0; i < k; ++i) {
      check_op(ctx, &cts[i], 2, "ciphertext");
      same_level(acc, &cts[i], "ciphertext");
      const ckks_operand cur{acc->data, acc->level, 2, sc};
      sc = product_scale(&cur, cts[i].scale * const_scale, "scalar_mul_acc");
      c[i] = cts[i].data;
    }
    const ficgcn_status st = ckks_scalar_mul_acc(ctx, acc->data, acc->level, c.data(), consts, k);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    acc->scale = sc;
  });
}

ficgcn_status ckks_add_op(ckks_ctx* ctx, ckks_operand* acc, const ckks_operand* in) {
  return guard([&] {
    check_op(ctx, acc, 2, "accumulator");
    check_op(ctx, in, 2, "ciphertext");
    same_level(acc, in, "ciphertext");
    REQUIRE(scale_eq(acc->scale, in->scale), ESCALE_,
            "add: scale " + std::to_string(in->scale) + " against " + std::to_string(acc->scale));
    const ficgcn_status st = ckks_add(ctx, acc->data, in->data, acc->level);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
  });
}

ficgcn_status ckks_rescale_op(ckks_ctx* ctx, ckks_operand* ct) {
  return guard([&] {
    check_op(ctx, ct, 2, "ciphertext");
    REQUIRE(ct->level >= 1, ELEVEL_, "rescale at level 0");
    const ficgcn_status st = ckks_rescale(ctx, ct->data, ct->level);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    ct->scale /= (double)ctx->mod[ct->level];
    ct->level -= 1;
  });
}

ficgcn_status ckks_mul_relin_op(ckks_ctx* ctx, const ckks_keys* eval_keys, const ckks_operand* x,
                                const ckks_operand* y, ckks_operand* out) {
  return guard([&] {
    check_op(ctx, x, 2, "x");
    check_op(ctx, y, 2, "y");
    same_level(x, y, "y");
    REQUIRE(out && out->data && out->n_poly == 2, EINVAL_, "output is not a ciphertext buffer");
    REQUIRE(out->level == x->level, ELEVEL_, "output is at another level");
    const ficgcn_status st = ckks_mul_relin(ctx, eval_keys, x->data, y->data, x->level, out->data);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
    out->scale = x->scale * y->scale;
  });
}

}  // extern "C"
