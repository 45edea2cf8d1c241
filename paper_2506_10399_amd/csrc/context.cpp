// CKKS context: prime chain, NTT twiddle tables, base-conversion constants.
//
// Prime chain (paper Sec. 2.1: Q = q_0 ... q_{L-1}): the L largest primes
// below 2^q_bits with q = 1 (mod 2N), in descending order, then the alpha
// largest primes below 2^p_bits with p = 1 (mod 2N) as the special modulus P
// of hybrid key switching.
#include <stdexcept>
#include <thread>

#include "internal.h"

namespace ficgcn {

uint64_t powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = (uint64_t)((u128)r * a % q);
    a = (uint64_t)((u128)a * a % q);
    e >>= 1;
  }
  return r;
}

uint64_t invmod(uint64_t a, uint64_t q) { return powmod(a, q - 2, q); }

uint64_t shoup(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }

Mod make_mod(uint64_t q) {
  // floor(2^128 / q) = floor((2^128 - 1) / q) for q not a power of two
  u128 all = ~(u128)0;
  u128 r = all / q;
  return Mod{q, (uint64_t)(r >> 64), (uint64_t)r};
}

static bool miller_rabin(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : bases)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = (uint64_t)((u128)x * x % n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

static std::vector<uint64_t> chain(int bits, int count, uint64_t two_n, const std::vector<uint64_t>& avoid) {
  std::vector<uint64_t> out;
  uint64_t top = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
  uint64_t p = top / two_n * two_n + 1;
  if (p > top) p -= two_n;
  while ((int)out.size() < count) {
    if (p < two_n) FICGCN_THROW(EINVAL_, "not enough NTT primes of this size");
    bool skip = false;
    for (uint64_t a : avoid) skip |= (a == p);
    if (!skip && miller_rabin(p)) out.push_back(p);
    p -= two_n;
  }
  return out;
}

static uint64_t root_2n(uint64_t q, uint64_t two_n) {
  uint64_t e = (q - 1) / two_n;
  for (uint64_t x = 2;; ++x) {
    uint64_t psi = powmod(x, e, q);
    if (powmod(psi, two_n / 2, q) == q - 1) return psi;
  }
}

static uint32_t brev_host(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

void build_context(ckks_ctx* c) {
  c->N = 1 << c->log_n;
  uint64_t two_n = 2ull * c->N;
  if (c->q_bits > 61 || c->p_bits > 61 || c->q_bits < 20 || c->p_bits < 20)
    FICGCN_THROW(EINVAL_, "prime sizes must be in [20, 61] bits");
  std::vector<uint64_t> q = chain(c->q_bits, c->L, two_n, {});
  std::vector<uint64_t> p = chain(c->p_bits, c->alpha, two_n, q);
  c->mod = q;
  c->mod.insert(c->mod.end(), p.begin(), p.end());
  int nm = c->n_mod();
  size_t N = c->N;
  std::vector<uint64_t> psi(nm * N), psi_s(nm * N), ipsi(nm * N), ipsi_s(nm * N), ninv(nm), ninv_s(nm);
  std::vector<Mod> mods(nm);
  c->psi.resize(nm);
  std::vector<std::thread> th;
  for (int m = 0; m < nm; ++m) {
    th.emplace_back([&, m]() {
      uint64_t qm = c->mod[m];
      uint64_t r = root_2n(qm, two_n);
      c->psi[m] = r;
      uint64_t ir = invmod(r, qm);
      // powers in natural order, then placed at bit-reversed positions
      std::vector<uint64_t> pw(N), ipw(N);
      pw[0] = 1;
      ipw[0] = 1;
      for (size_t k = 1; k < N; ++k) {
        pw[k] = (uint64_t)((u128)pw[k - 1] * r % qm);
        ipw[k] = (uint64_t)((u128)ipw[k - 1] * ir % qm);
      }
      for (size_t k = 0; k < N; ++k) {
        uint32_t b = brev_host((uint32_t)k, c->log_n);
        psi[m * N + k] = pw[b];
        psi_s[m * N + k] = shoup(pw[b], qm);
        ipsi[m * N + k] = ipw[b];
        ipsi_s[m * N + k] = shoup(ipw[b], qm);
      }
      ninv[m] = invmod(N % qm, qm);
      ninv_s[m] = shoup(ninv[m], qm);
      mods[m] = make_mod(qm);
    });
  }
  for (auto& t : th) t.join();
  c->h_psi.swap(psi);
  c->h_psi_s.swap(psi_s);
  c->h_ipsi.swap(ipsi);
  c->h_ipsi_s.swap(ipsi_s);
  c->h_ninv.swap(ninv);
  c->h_ninv_s.swap(ninv_s);
  c->h_mods.swap(mods);
}

void ensure_device(ckks_ctx* c) {
  if (c->on_device) return;
  HIPCHECK(hipGetDevice(&c->device));
  auto up = [&](uint64_t** dst, const std::vector<uint64_t>& v) {
    HIPCHECK(hipMalloc(dst, v.size() * 8));
    HIPCHECK(hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice));
  };
  up(&c->t.psi, c->h_psi);
  up(&c->t.psi_s, c->h_psi_s);
  up(&c->t.ipsi, c->h_ipsi);
  up(&c->t.ipsi_s, c->h_ipsi_s);
  auto up_f = [&](double** dst, const std::vector<uint64_t>& v) {
    std::vector<double> f(v.size());
    for (size_t i = 0; i < v.size(); ++i) f[i] = (double)v[i];
    HIPCHECK(hipMalloc(dst, f.size() * 8));
    HIPCHECK(hipMemcpy(*dst, f.data(), f.size() * 8, hipMemcpyHostToDevice));
  };
  up_f(&c->t.psi_f, c->h_psi);
  up_f(&c->t.ipsi_f, c->h_ipsi);
  up(&c->t.ninv, c->h_ninv);
  up(&c->t.ninv_s, c->h_ninv_s);
  HIPCHECK(hipMalloc(&c->t.mods, c->h_mods.size() * sizeof(Mod)));
  HIPCHECK(hipMemcpy(c->t.mods, c->h_mods.data(), c->h_mods.size() * sizeof(Mod), hipMemcpyHostToDevice));
  c->on_device = true;
  // every base-conversion table of the chain, so later calls find them built
  for (int level = 0; level < c->L; ++level) {
    for (int d = 0; d * c->alpha <= level; ++d) get_modup(c, level, d);
    get_moddown(c, level);
  }
}

// FastBConv constants: hat_b = prod_{s' != s} b_{s'}; hat_inv[s] = hat_b^-1 mod b_s;
// hat_mod[d][s] = hat_b mod p_d.
static BConv make_bconv(ckks_ctx* c, const std::vector<int>& src, const std::vector<int>& dst) {
  BConv bc;
  bc.src = src;
  bc.dst = dst;
  bc.n_src = (int)src.size();
  bc.n_dst = (int)dst.size();
  std::vector<uint64_t> h(2 * bc.n_src + bc.n_dst * bc.n_src);
  for (int s = 0; s < bc.n_src; ++s) {
    uint64_t bs = c->mod[src[s]];
    uint64_t hat = 1;
    for (int s2 = 0; s2 < bc.n_src; ++s2)
      if (s2 != s) hat = (uint64_t)((u128)hat * (c->mod[src[s2]] % bs) % bs);
    h[s] = invmod(hat, bs);
    h[bc.n_src + s] = shoup(h[s], bs);
  }
  for (int d = 0; d < bc.n_dst; ++d) {
    uint64_t pd = c->mod[dst[d]];
    for (int s = 0; s < bc.n_src; ++s) {
      uint64_t hat = 1;
      for (int s2 = 0; s2 < bc.n_src; ++s2)
        if (s2 != s) hat = (uint64_t)((u128)hat * (c->mod[src[s2]] % pd) % pd);
      h[2 * bc.n_src + d * bc.n_src + s] = hat;
    }
  }
  HIPCHECK(hipMalloc(&bc.dev, h.size() * 8));
  HIPCHECK(hipMemcpy(bc.dev, h.data(), h.size() * 8, hipMemcpyHostToDevice));
  std::vector<int> ix(src);
  ix.insert(ix.end(), dst.begin(), dst.end());
  HIPCHECK(hipMalloc(&bc.idx, ix.size() * sizeof(int)));
  HIPCHECK(hipMemcpy(bc.idx, ix.data(), ix.size() * sizeof(int), hipMemcpyHostToDevice));
  return bc;
}

// ModUp of digit `digit` at `level`: source = the digit's active Q primes,
// destinations = every other active Q prime, then the P primes.
const BConv& get_modup(ckks_ctx* c, int level, int digit) {
  auto key = std::make_pair(level, digit);
  auto it = c->modup.find(key);
  if (it != c->modup.end()) return it->second;
  std::vector<int> src, dst;
  int lo = digit * c->alpha, hi = std::min((digit + 1) * c->alpha, level + 1);
  for (int i = lo; i < hi; ++i) src.push_back(i);
  for (int i = 0; i <= level; ++i)
    if (i < lo || i >= hi) dst.push_back(i);
  for (int k = 0; k < c->alpha; ++k) dst.push_back(c->L + k);
  return c->modup[key] = make_bconv(c, src, dst);
}

const BConv& get_moddown(ckks_ctx* c, int level) {
  auto it = c->moddown.find(level);
  if (it != c->moddown.end()) return it->second;
  std::vector<int> src, dst;
  for (int k = 0; k < c->alpha; ++k) src.push_back(c->L + k);
  for (int i = 0; i <= level; ++i) dst.push_back(i);
  return c->moddown[level] = make_bconv(c, src, dst);
}

uint64_t galois_elt(ckks_ctx* c, int64_t step) {
  int64_t M = c->N / 2;
  int64_t k = ((step % M) + M) % M;
  return powmod(5, (uint64_t)k, 2ull * c->N);
}

}  // namespace ficgcn

namespace ficgcn {

Recorder::~Recorder() {
  for (auto& b : bufs)
    if (b.first) (void)hipFree(b.first);
}

static void* recorded(ckks_ctx* c, size_t bytes, const void* host) {
  Recorder* r = c->rec;
  if (r->mode == Recorder::RECORD) {
    void* d = nullptr;
    HIPCHECK(hipMalloc(&d, std::max<size_t>(16, bytes)));
    r->bufs.push_back({d, bytes});
    if (host && bytes) {
      HIPCHECK(hipStreamSynchronize(c->stream));
      HIPCHECK(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
    }
    return d;
  }
  if (r->cursor >= r->bufs.size() || r->bufs[r->cursor].second != bytes)
    FICGCN_THROW(EPLAN_, "replayed launch sequence differs from the recorded one");
  return r->bufs[r->cursor++].first;
}

void* dev_scratch(ckks_ctx* c, int slot, size_t bytes) {
  if (c->rec) return recorded(c, bytes, nullptr);
  return c->buf(slot, bytes);
}

void* dev_table(ckks_ctx* c, int slot, const void* host, size_t bytes) {
  if (c->rec) return recorded(c, bytes, host);
  void* d = c->buf(slot, std::max<size_t>(16, bytes));
  if (bytes) HIPCHECK(hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, c->stream));
  return d;
}

void stream_sync(ckks_ctx* c) {
  if (c->rec && c->rec->mode == Recorder::REPLAY) return;
  HIPCHECK(hipStreamSynchronize(c->stream));
}

}  // namespace ficgcn

void* ckks_ctx::buf(int slot, size_t bytes) {
  if ((int)scratch.size() <= slot) scratch.resize(slot + 1, {nullptr, 0});
  auto& s = scratch[slot];
  if (s.second < bytes) {
    if (s.first) {
      HIPCHECK(hipStreamSynchronize(stream));
      HIPCHECK(hipFree(s.first));
    }
    s.first = nullptr;
    HIPCHECK(hipMalloc(&s.first, bytes));
    s.second = bytes;
  }
  return s.first;
}

ckks_ctx::~ckks_ctx() {
  if (stream) (void)hipStreamSynchronize(stream);
  for (auto& s : scratch)
    if (s.first) (void)hipFree(s.first);
  for (uint64_t* p : {t.psi, t.psi_s, t.ipsi, t.ipsi_s, t.ninv, t.ninv_s})
    if (p) (void)hipFree(p);
  for (double* p : {t.psi_f, t.ipsi_f, enc_root, enc_twist})
    if (p) (void)hipFree(p);
  if (enc_pos) (void)hipFree(enc_pos);
  if (enc_flag) (void)hipFree(enc_flag);
  if (t.mods) (void)hipFree(t.mods);
  for (auto& kv : modup) { (void)hipFree(kv.second.dev); (void)hipFree(kv.second.idx); }
  for (auto& kv : moddown) { (void)hipFree(kv.second.dev); (void)hipFree(kv.second.idx); }
}

ckks_keys::~ckks_keys() {
  if (ctx && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (s_ntt) (void)hipFree(s_ntt);
  for (auto& kv : swk) (void)hipFree(kv.second);
}
