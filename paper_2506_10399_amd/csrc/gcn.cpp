// GCN layer executor and the plan entry points.
//
// A layer runs in one of two forms that produce identical words:
//  plain   (mode 0): one HE operation per library call -- PMult/Add per
//          Inter-CA copy, scalar MAC per weight, one key switch (ModUp,
//          inner product, ModDown) per rotation, one rescale per ciphertext;
//  batched (mode 1): the Inter-CA aggregation and the combination fused in
//          one pass over the inputs; the rotations of each stage (packing,
//          baby steps, giant steps, the diagonal shifts) and the
//          relinearisations of a layer run as one key-switch batch, the
//          rotations of a source hoisted on one ModUp and the masked sums
//          folded into the batch's final ModDown step; rescales batched.
// Words agree because every step is exact modular arithmetic and a rotation
// is defined as ModUp, automorphism, inner product, ModDown in both forms.
#include <algorithm>
#include <cstring>
#include <map>
#include <set>

#include "../../include/ficgcn.h"
#include "ks_batch.h"
#include "plan.h"

namespace ficgcn {

void comb_fused(ckks_ctx* c, const std::vector<uint64_t*>& outs, const uint64_t* in_base, size_t in_stride,
                const uint64_t* const* in_dev_ptrs, const PtrList& pts, int K, int F, int F_out, int level,
                const void* w_dev, bool split, const char* prof_name);
void zero_fill(ckks_ctx* c, uint64_t* p, size_t words);
bool mfma_supported(ckks_ctx* c, int K, int F, int F_out);
bool mfma_weight_planes(const std::vector<int64_t>& w_int, int F, int F_out, int l0, std::vector<uint8_t>& planes,
                        int& n_fb);
void mfma_pow256(ckks_ctx* c, int l1, std::vector<uint64_t>& out);
size_t mfma_packed_words(ckks_ctx* c, int K, int F, int level);
bool mfma_pack_supported(ckks_ctx* c);
void mfma_pack(ckks_ctx* c, const uint64_t* in_base, size_t in_stride, const uint64_t* const* in_ptrs, int K, int F,
               int level, uint64_t* packed);
void comb_mfma_packed(ckks_ctx* c, const std::vector<uint64_t*>& outs, const uint64_t* packed, const PtrList& pts, int K,
                      int F, int level, const void* wd, const uint64_t* pw, const char* prof_name);
void comb_mfma(ckks_ctx* c, const std::vector<uint64_t*>& outs, const uint64_t* in_base, size_t in_stride,
               const uint64_t* const* in_dev_ptrs, const PtrList& pts, int K, int F, int level, const void* wd,
               const uint64_t* pw, const char* prof_name);
void build_plan(ckks_ctx* c, ficgcn_plan* p, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                const ficgcn_plan_opts& o);

static int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}
static int64_t fmodp(int64_t a, int64_t b) { return a - fdiv(a, b) * b; }

static uint64_t residue(int64_t v, uint64_t q) {
  return v >= 0 ? (uint64_t)v % q : (q - (uint64_t)(-(v + 1)) % q - 1) % q;
}

// weights as [F'][F][l1][2] (residue, Shoup) at the combination level
static void ensure_weights(ckks_ctx* c, LayerPlan& lp) {
  if (lp.w_dev) return;
  const int l1 = lp.level_in + 1;
  std::vector<uint64_t> h((size_t)lp.f_out * lp.f_in * l1 * 2);
  for (int l = 0; l < lp.f_out; ++l)
    for (int f = 0; f < lp.f_in; ++f)
      for (int i = 0; i < l1; ++i) {
        uint64_t q = c->mod[i];
        uint64_t r = residue(lp.w_int[(size_t)f * lp.f_out + l], q);
        size_t o = (((size_t)l * lp.f_in + f) * l1 + i) * 2;
        h[o] = r;
        h[o + 1] = shoup(r, q);
      }
  HIPCHECK(hipMalloc(&lp.w_dev, h.size() * 8));
  HIPCHECK(hipMemcpy(lp.w_dev, h.data(), h.size() * 8, hipMemcpyHostToDevice));
}

// weights of the fused pass, [l1][F][F'] in the form the kernel reads:
// 26-bit halves (uint32 pairs) when every active prime is below 2^52, else residues
static void ensure_fused_weights(ckks_ctx* c, LayerPlan& lp) {
  if (lp.wf_dev) return;
  const int l1 = lp.level_in + 1;
  lp.wf_split = c->mod[0] < (1ull << 52);
  const size_t n = (size_t)l1 * lp.f_in * lp.f_out;
  if (lp.wf_split) {
    const int F_pad = (lp.f_out + 15) / 16 * 16;   // zero columns up to the kernel's unroll width
    std::vector<uint32_t> h((size_t)2 * l1 * lp.f_in * F_pad, 0u);
    for (int i = 0; i < l1; ++i)
      for (int f = 0; f < lp.f_in; ++f)
        for (int l = 0; l < lp.f_out; ++l) {
          uint64_t r = residue(lp.w_int[(size_t)f * lp.f_out + l], c->mod[i]);
          size_t o = (((size_t)i * lp.f_in + f) * F_pad + l) * 2;
          h[o] = (uint32_t)(r & ((1u << 26) - 1));
          h[o + 1] = (uint32_t)(r >> 26);
        }
    HIPCHECK(hipMalloc(&lp.wf_dev, h.size() * 4));
    HIPCHECK(hipMemcpy(lp.wf_dev, h.data(), h.size() * 4, hipMemcpyHostToDevice));
  } else {
    std::vector<uint64_t> h(n);
    for (int i = 0; i < l1; ++i)
      for (int f = 0; f < lp.f_in; ++f)
        for (int l = 0; l < lp.f_out; ++l)
          h[((size_t)i * lp.f_in + f) * lp.f_out + l] = residue(lp.w_int[(size_t)f * lp.f_out + l], c->mod[i]);
    HIPCHECK(hipMalloc(&lp.wf_dev, h.size() * 8));
    HIPCHECK(hipMemcpy(lp.wf_dev, h.data(), h.size() * 8, hipMemcpyHostToDevice));
  }
}

// Digit planes of the weights for the matrix-core pass; false when the
// layer's shape or weights are outside it (the split pass runs instead).
static bool ensure_mfma_weights(ckks_ctx* c, LayerPlan& lp, int K) {
  if (lp.wm_state) return lp.wm_state > 0;
  lp.wm_state = -1;
  if (!mfma_supported(c, K, lp.f_in, std::min(lp.f_out, 16))) return false;
  const int groups = (lp.f_out + 15) / 16;
  std::vector<uint8_t> all, one;
  int n_fb = 0;
  for (int gi = 0; gi < groups; ++gi) {
    if (!mfma_weight_planes(lp.w_int, lp.f_in, lp.f_out, gi * 16, one, n_fb)) return false;
    all.insert(all.end(), one.begin(), one.end());
  }
  lp.wm_group_bytes = one.size();
  std::vector<uint64_t> pw;
  mfma_pow256(c, lp.level_in + 1, pw);
  HIPCHECK(hipMalloc(&lp.wm_dev, all.size()));
  HIPCHECK(hipMemcpy(lp.wm_dev, all.data(), all.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMalloc(&lp.pw_dev, pw.size() * 8));
  HIPCHECK(hipMemcpy(lp.pw_dev, pw.data(), pw.size() * 8, hipMemcpyHostToDevice));
  lp.wm_state = 1;
  return true;
}

// Every table the layers build on first use (per-operation weights, the fused passes'
// weights and digit planes), built now: afterwards running the plan only reads it.
void prepare_plan_device(ckks_ctx* c, ficgcn_plan* p) {
  for (LayerPlan& lp : p->layers) {
    ensure_weights(c, lp);
    ensure_fused_weights(c, lp);
    if (lp.kind == 0) ensure_mfma_weights(c, lp, lp.K);
    for (size_t i = 0; i < lp.ops.size(); ++i)
      if (!lp.ops[i] && lp.op_alias[i] >= 0) lp.ops[i] = lp.ops[lp.op_alias[i]];
  }
}

// Fused pass of one layer on its rearranged inputs (matrix-core form only)
static void fused_pass_packed(ckks_ctx* c, LayerPlan& lp, const std::vector<uint64_t*>& outs, const PtrList& pts, int K,
                              const char* name) {
  if (!lp.packed_in || !ensure_mfma_weights(c, lp, K)) FICGCN_THROW(EPLAN_, "no rearranged inputs for this layer");
  for (int l0 = 0; l0 < lp.f_out; l0 += 16) {
    std::vector<uint64_t*> o(outs.begin() + l0, outs.begin() + std::min(lp.f_out, l0 + 16));
    comb_mfma_packed(c, o, lp.packed_in, pts, K, lp.f_in, lp.level_in,
                     lp.wm_dev + (size_t)(l0 / 16) * lp.wm_group_bytes, lp.pw_dev, name);
  }
}

// Fused pass of one layer: matrix-core form where it applies, else the split form
static void fused_pass(ckks_ctx* c, LayerPlan& lp, const std::vector<uint64_t*>& outs, const uint64_t* base,
                       size_t stride, const uint64_t* const* idv, const PtrList& pts, int K, const char* name) {
  // buffer loads address a 64-ciphertext span with 31-bit offsets
  if (ensure_mfma_weights(c, lp, K) && (!base || stride < ((size_t)1 << 22))) {
    for (int l0 = 0; l0 < lp.f_out; l0 += 16) {
      std::vector<uint64_t*> o(outs.begin() + l0, outs.begin() + std::min(lp.f_out, l0 + 16));
      comb_mfma(c, o, base, stride, idv, pts, K, lp.f_in, lp.level_in, lp.wm_dev + (size_t)(l0 / 16) * lp.wm_group_bytes,
                lp.pw_dev, name);
    }
    return;
  }
  ensure_fused_weights(c, lp);
  comb_fused(c, outs, base, stride, idv, pts, K, lp.f_in, lp.f_out, lp.level_in, lp.wf_dev, lp.wf_split, name);
}

// A batch of equally spaced buffers is read by base + stride (no pointer table).
static bool strided(const uint64_t* const* p, size_t n, size_t min_words, const uint64_t*& base, size_t& stride) {
  base = p[0];
  if (n == 1) {
    stride = min_words;
    return true;
  }
  if (p[1] <= p[0]) return false;
  stride = (size_t)(p[1] - p[0]);
  if (stride < min_words) return false;
  for (size_t i = 2; i < n; ++i)
    if (p[i] != p[0] + i * stride) return false;
  return true;
}

template <typename T>
static T* upload_ptrs(ckks_ctx* c, const std::vector<T>& v, int slot) {
  T* d = (T*)dev_table(c, slot, v.data(), v.size() * sizeof(T));
  stream_sync(c);
  return d;
}

static const uint64_t* rot_key(ckks_ctx* c, const ckks_keys* ek, int64_t step, uint64_t& g);

// one key switch of a whole ciphertext (non-hoisted), out != in
static void rotate_one(ckks_ctx* c, const ckks_keys* ek, const uint64_t* in, int level, int64_t step, uint64_t* out) {
  const size_t N = c->N;
  const int l1 = level + 1, ext = l1 + c->alpha;
  const int nd = (l1 + c->alpha - 1) / c->alpha;
  uint64_t g = galois_elt(c, step);
  if (g == 1) {
    copy_d2d(c, out, in, (size_t)2 * l1 * N * 8);
    return;
  }
  auto it = ek->swk.find(g);
  if (it == ek->swk.end()) FICGCN_THROW(ENOKEY_, "missing rotation key for step " + std::to_string(step));
  uint64_t* D = (uint64_t*)c->buf(40, (size_t)nd * ext * N * 8);
  uint64_t* acc = (uint64_t*)c->buf(41, (size_t)2 * ext * N * 8);
  modup(c, in + (size_t)l1 * N, level, D);
  keymac(c, acc, D, it->second, level, g);
  moddown(c, acc, level, out, in, g, nullptr);
}

// Radix-2 program (family 3) of one packed ciphertext, one operation per
// call: per step and rotation amount one key switch, then the masks of that
// amount into the next registers and the result terms.  Registers are
// accumulated at their step's level and rescaled when first read; result
// terms (one per level) are rescaled, dropped to the output level and summed.
static void aggregate_r2_plain(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, int g, const uint64_t* y,
                               uint64_t* out) {
  const size_t N = c->N;
  const R2Program& pr = lp.r2;
  const int la = lp.level_agg, D = pr.depth, lo = la - D;
  const size_t nops = pr.ops.size();
  auto mask = [&](size_t j) { return (const uint64_t*)lp.ops[(size_t)g * nops + j]; };
  auto ctw = [&](int level) { return (size_t)2 * (level + 1) * N; };
  const int nreg = (int)pr.reg_depth.size();
  std::vector<size_t> roff(nreg, 0), ooff(D, 0);
  size_t rtot = 0, otot = 0;
  for (int r = 1; r < nreg; ++r) {
    roff[r] = rtot;
    rtot += ctw(la - pr.reg_depth[r] + 1);
  }
  for (int d = 0; d < D; ++d) {
    ooff[d] = otot;
    otot += ctw(la - d);
  }
  uint64_t* regs = (uint64_t*)c->buf(75, std::max<size_t>(1, rtot) * 8);
  uint64_t* obuf = (uint64_t*)c->buf(76, otot * 8);
  uint64_t* rt = (uint64_t*)c->buf(77, ctw(la) * 8);
  if (rtot) zero_fill(c, regs, rtot);
  zero_fill(c, obuf, otot);
  std::vector<char> ready(nreg, 0);
  ready[0] = 1;
  auto reg = [&](int r) -> const uint64_t* {
    if (r == 0) return y;
    if (!ready[r]) {
      rescale_inplace(c, regs + roff[r], la - pr.reg_depth[r] + 1);
      ready[r] = 1;
    }
    return regs + roff[r];
  };
  auto mac = [&](uint64_t* acc, const uint64_t* ct, const uint64_t* pt, int l1) {
    PtrList a{}, b{};
    a.p[0] = ct;
    b.p[0] = pt;
    pmul_acc(c, acc, a, b, 1, l1);
  };
  mac(obuf + ooff[0], y, mask(0), la + 1);
  size_t j0 = 1;
  for (const R2Step& st : pr.steps) {
    const int level = la - st.depth, l1 = level + 1;
    const uint64_t* src = reg(st.src);
    std::set<int64_t> ms;
    for (const R2Term& t : st.keep) ms.insert(t.m);
    for (const R2Term& t : st.fin) ms.insert(t.m);
    const size_t nk = st.keep.size();
    for (int64_t m : ms) {
      const uint64_t* rm = src;
      if (m != 0) {
        rotate_one(c, ek, src, level, m, rt);
        rm = rt;
      }
      for (size_t t = 0; t < nk; ++t)
        if (st.keep[t].m == m) mac(regs + roff[st.keep[t].dst], rm, mask(j0 + t), l1);
      for (size_t t = 0; t < st.fin.size(); ++t)
        if (st.fin[t].m == m) mac(obuf + ooff[st.depth], rm, mask(j0 + nk + t), l1);
    }
    j0 += nk + st.fin.size();
  }
  zero_fill(c, out, ctw(lo));
  for (int d = 0; d < D; ++d) {
    uint64_t* o = obuf + ooff[d];
    rescale_inplace(c, o, la - d);                   // now [2][la - d][N]
    add_inplace(c, out, o, lo + 1, 1);
    add_inplace(c, out + (size_t)(lo + 1) * N, o + (size_t)(la - d) * N, lo + 1, 1);
  }
}

// SpIntra-CA of one packed ciphertext, one operation per call (plain form)
// Double-hoisted diagonal form (family 4) of one packed ciphertext, one
// operation per call: one ModUp of y's c1; per nonzero shift the key inner
// product of the automorphed digits, multiplied by the mask on the key basis
// and summed, and sigma(c0) (.) mask summed on Q_l; one ModDown of the sum;
// the identity shift's plain mask product; rescale.
// out = sum_k Rot_{steps[k]}(y) (.) masks[k] at level lv, one operation per call: the nonzero
// steps' key inner products times their masks summed on the key basis (masks of those steps
// hold level+1+alpha limbs), one ModDown; a zero step is a plain mask product.  No rescale.
static void masked_sum_plain(ckks_ctx* c, const ckks_keys* ek, const uint64_t* y, int lv,
                             const std::vector<int64_t>& steps, const std::vector<const uint64_t*>& masks,
                             uint64_t* out) {
  const size_t N = c->N;
  const int l1 = lv + 1, ext = l1 + c->alpha;
  const int nd = (l1 + c->alpha - 1) / c->alpha;
  const size_t ns = steps.size();
  auto mask = [&](size_t si) { return masks[si]; };
  uint64_t* D = (uint64_t*)c->buf(40, (size_t)nd * ext * N * 8);
  uint64_t* acc = (uint64_t*)c->buf(41, (size_t)2 * ext * N * 8);
  uint64_t* A = (uint64_t*)c->buf(78, (size_t)2 * ext * N * 8);
  uint64_t* t = (uint64_t*)c->buf(79, (size_t)2 * l1 * N * 8);   // (sigma(c0), 0)
  zero_fill(c, A, (size_t)2 * ext * N);
  zero_fill(c, out, (size_t)2 * l1 * N);
  zero_fill(c, t + (size_t)l1 * N, (size_t)l1 * N);
  modup(c, y + (size_t)l1 * N, lv, D);
  auto mac = [&](const uint64_t* ct, const uint64_t* pt) {
    PtrList a{}, b{};
    a.p[0] = ct;
    b.p[0] = pt;
    pmul_acc(c, out, a, b, 1, l1);
  };
  for (size_t si = 0; si < ns; ++si) {
    const int64_t d = steps[si];
    uint64_t gal;
    const uint64_t* key = rot_key(c, ek, d, gal);
    if (!key) {
      mac(y, mask(si));
      continue;
    }
    keymac(c, acc, D, key, lv, gal);
    mac_ext(c, A, acc, mask(si), lv);
    automorph_ntt(c, t, y, gal, l1, 1);
    mac(t, mask(si));
  }
  uint64_t* md = (uint64_t*)c->buf(44, (size_t)2 * l1 * N * 8);
  moddown(c, A, lv, md, nullptr, 1, nullptr);
  add_inplace(c, out, md, l1, 2);
}

static void aggregate_dh_plain(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, int g, const uint64_t* y,
                               uint64_t* out) {
  const size_t ns = lp.shifts.size();
  std::vector<const uint64_t*> masks(ns);
  for (size_t si = 0; si < ns; ++si) masks[si] = lp.ops[(size_t)g * ns + si];
  masked_sum_plain(c, ek, y, lp.level_agg, lp.shifts, masks, out);
  rescale_inplace(c, out, lp.level_agg);
}

static void aggregate(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, int g, const uint64_t* y, uint64_t* out) {
  if (lp.family == 3) {
    aggregate_r2_plain(c, ek, lp, g, y, out);
    return;
  }
  if (lp.family == 4) {
    aggregate_dh_plain(c, ek, lp, g, y, out);
    return;
  }
  const size_t N = c->N;
  const int lv = lp.level_agg, l1 = lv + 1;
  const size_t ct_words = (size_t)2 * l1 * N;
  const size_t ns = lp.shifts.size();
  uint64_t* rt = (uint64_t*)c->buf(44, ct_words * 8);
  zero_fill(c, out, ct_words);
  auto mask = [&](size_t si) { return (const uint64_t*)lp.ops[(size_t)g * ns + si]; };
  auto mac = [&](const uint64_t* ct, const uint64_t* pt) {
    PtrList a{}, b{};
    a.p[0] = ct;
    b.p[0] = pt;
    pmul_acc(c, out, a, b, 1, l1);
  };
  if (lp.family == 1) {
    for (size_t si = 0; si < ns; ++si) {
      int64_t d = lp.shifts[si];
      if (d == 0) {
        mac(y, mask(si));
        continue;
      }
      rotate_one(c, ek, y, lv, d, rt);
      mac(rt, mask(si));
    }
  } else {
    const int64_t G = lp.G;
    std::set<int64_t> babies;
    std::map<int64_t, std::vector<size_t>> giants;
    for (size_t si = 0; si < ns; ++si) {
      int64_t d = lp.shifts[si];
      if (fmodp(d, G)) babies.insert(fmodp(d, G));
      giants[fdiv(d, G)].push_back(si);
    }
    // baby rotations of y, kept for every giant step
    std::map<int64_t, uint64_t*> rb;
    uint64_t* bb = (uint64_t*)c->buf(45, std::max<size_t>(1, babies.size()) * ct_words * 8);
    size_t bi = 0;
    for (int64_t b : babies) {
      uint64_t* dst = bb + (bi++) * ct_words;
      rotate_one(c, ek, y, lv, b, dst);
      rb[b] = dst;
    }
    // giant rotations: Sum_gi Rot_{gi G}(inner_gi) with one ModDown,
    //   out += ModDown(Sum KeyInner(sigma(ModUp(inner_gi.c1)))) + Sum sigma(inner_gi.c0)
    const int ext = l1 + c->alpha;
    const int nd = (l1 + c->alpha - 1) / c->alpha;
    uint64_t* inner = (uint64_t*)c->buf(46, ct_words * 8);
    uint64_t* D = (uint64_t*)c->buf(40, (size_t)nd * ext * N * 8);
    uint64_t* acc = (uint64_t*)c->buf(41, (size_t)2 * ext * N * 8);
    uint64_t* A = (uint64_t*)c->buf(78, (size_t)2 * ext * N * 8);
    uint64_t* t = (uint64_t*)c->buf(79, ct_words * 8);   // (sigma(c0), 0)
    bool any = false;
    for (auto& kv : giants) {
      int64_t gi = kv.first;
      zero_fill(c, inner, ct_words);
      for (size_t si : kv.second) {
        int64_t b = fmodp(lp.shifts[si], G);
        PtrList a{}, m{};
        a.p[0] = b ? rb[b] : y;
        m.p[0] = mask(si);
        pmul_acc(c, inner, a, m, 1, l1);
      }
      uint64_t gal;
      const uint64_t* key = gi != 0 ? rot_key(c, ek, gi * G, gal) : nullptr;
      if (!key) {
        add_inplace(c, out, inner, l1, 2);
        continue;
      }
      if (!any) {
        zero_fill(c, A, (size_t)2 * ext * N);
        zero_fill(c, t + (size_t)l1 * N, (size_t)l1 * N);
        any = true;
      }
      modup(c, inner + (size_t)l1 * N, lv, D);
      keymac(c, acc, D, key, lv, gal);
      mac_ext(c, A, acc, nullptr, lv);
      automorph_ntt(c, t, inner, gal, l1, 1);
      add_inplace(c, out, t, l1, 2);
    }
    if (any) {
      uint64_t* md = (uint64_t*)c->buf(44, ct_words * 8);
      moddown(c, A, lv, md, nullptr, 1, nullptr);
      add_inplace(c, out, md, l1, 2);
    }
  }
  rescale_inplace(c, out, lv);
}

// Galois element and switching key of a rotation step; null key for the identity
static const uint64_t* rot_key(ckks_ctx* c, const ckks_keys* ek, int64_t step, uint64_t& g) {
  g = galois_elt(c, step);
  if (g == 1) return nullptr;
  auto it = ek->swk.find(g);
  if (it == ek->swk.end()) FICGCN_THROW(ENOKEY_, "missing rotation key for step " + std::to_string(step));
  return it->second;
}

// Radix-2 program (family 3) of every packed ciphertext (batched form).
// Steps are taken boundary by boundary (the rounds they start at) and, within
// a boundary, level by level: one key-switch batch for the distinct
// (register, amount) rotations of every packed ciphertext, one masked-sum
// launch into the next registers, one into the result terms; the registers
// written at a boundary are rescaled together.  The result terms are rescaled
// and summed into the outputs at the output level.
static void aggregate_r2_batched(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, const std::vector<uint64_t*>& Y,
                                 const std::vector<uint64_t*>& outs) {
  const size_t N = c->N;
  const R2Program& pr = lp.r2;
  const int la = lp.level_agg, D = pr.depth, lo = la - D;
  const int np = (int)Y.size();
  const size_t nops = pr.ops.size();
  auto mask = [&](int g, size_t j) { return (const uint64_t*)lp.ops[(size_t)g * nops + j]; };
  auto ctw = [&](int level) { return (size_t)2 * (level + 1) * N; };
  const int nreg = (int)pr.reg_depth.size();
  std::vector<size_t> roff(nreg, 0), ooff(D, 0);
  size_t RB = 0, OB = 0;
  for (int r = 1; r < nreg; ++r) {
    roff[r] = RB;
    RB += ctw(la - pr.reg_depth[r] + 1);
  }
  for (int d = 0; d < D; ++d) {
    ooff[d] = OB;
    OB += ctw(la - d);
  }
  // operand index of each step's first term
  std::vector<size_t> first(pr.steps.size());
  {
    size_t j = 1;
    for (size_t s = 0; s < pr.steps.size(); ++s) {
      first[s] = j;
      j += pr.steps[s].keep.size() + pr.steps[s].fin.size();
    }
  }
  // (boundary, depth) groups in program order, and the largest rotation set
  std::vector<std::pair<size_t, size_t>> runs;   // [begin, end) of equal r0
  for (size_t s = 0; s < pr.steps.size();) {
    size_t e = s;
    while (e < pr.steps.size() && pr.steps[e].r0 == pr.steps[s].r0) ++e;
    runs.push_back({s, e});
    s = e;
  }
  size_t max_rot = 1;
  for (auto& rn : runs) {
    std::map<int, std::set<std::pair<int, int64_t>>> per_depth;
    for (size_t s = rn.first; s < rn.second; ++s) {
      const R2Step& st = pr.steps[s];
      for (const auto* v : {&st.keep, &st.fin})
        for (const R2Term& t : *v)
          if (t.m) per_depth[st.depth].insert({st.src, t.m});
    }
    for (auto& kv : per_depth) max_rot = std::max(max_rot, kv.second.size());
  }
  uint64_t* regs = (uint64_t*)dev_scratch(c, 72, std::max<size_t>(1, (size_t)np * RB) * 8);
  uint64_t* obuf = (uint64_t*)dev_scratch(c, 73, (size_t)np * OB * 8);
  uint64_t* rbuf = (uint64_t*)dev_scratch(c, 74, (size_t)np * max_rot * ctw(la) * 8);
  zero_fill(c, obuf, (size_t)np * OB);
  auto reg = [&](int g, int r) -> uint64_t* { return r == 0 ? Y[g] : regs + (size_t)g * RB + roff[r]; };
  auto oterm = [&](int g, int d) { return obuf + (size_t)g * OB + ooff[d]; };
  {
    std::vector<std::vector<MacTerm>> grp(np);
    std::vector<uint64_t*> go(np);
    for (int g = 0; g < np; ++g) {
      grp[g].push_back(MacTerm{Y[g], mask(g, 0)});
      go[g] = oterm(g, 0);
    }
    group_mac(c, la, grp, go, true);
  }
  for (auto& rn : runs) {
    std::map<int, std::vector<size_t>> by_depth;
    for (size_t s = rn.first; s < rn.second; ++s) by_depth[pr.steps[s].depth].push_back(s);
    std::map<int, std::vector<int>> written;          // depth -> registers written at this boundary
    for (auto& kv : by_depth) {
      const int d = kv.first, level = la - d;
      const size_t w = ctw(level);
      // distinct rotations of this level's steps
      // numbered in (register, amount) order, so the key-switch jobs come sorted by output
      std::map<std::pair<int, int64_t>, int> rix;
      std::map<int, int> six;
      for (size_t s : kv.second) {
        const R2Step& st = pr.steps[s];
        for (const auto* v : {&st.keep, &st.fin})
          for (const R2Term& t : *v)
            if (t.m) rix.emplace(std::make_pair(st.src, t.m), 0);
      }
      {
        int k = 0;
        for (auto& kv2 : rix) {
          kv2.second = k++;
          if (!six.count(kv2.first.first)) six.emplace(kv2.first.first, (int)six.size());
        }
      }
      const int nr = (int)rix.size(), ns = (int)six.size();
      auto rot = [&](int g, int src, int64_t m) -> const uint64_t* {
        if (m == 0) return reg(g, src);
        return rbuf + ((size_t)g * nr + rix.at({src, m})) * w;
      };
      if (nr) {
        std::vector<const uint64_t*> sources((size_t)np * ns);
        for (int g = 0; g < np; ++g)
          for (auto& sv : six) sources[(size_t)g * ns + sv.second] = reg(g, sv.first) + (size_t)(level + 1) * N;
        std::vector<KSJob> jobs;
        std::vector<uint64_t*> routs((size_t)np * nr);
        for (int g = 0; g < np; ++g)
          for (auto& kv2 : rix) {
            uint64_t gal;
            const uint64_t* key = rot_key(c, ek, kv2.first.second, gal);
            const int k = g * nr + kv2.second;
            routs[k] = rbuf + (size_t)k * w;
            jobs.push_back(KSJob{key, reg(g, kv2.first.first), nullptr, nullptr, gal,
                                 g * ns + six.at(kv2.first.first), k});
          }
        keyswitch_batch(c, level, sources, jobs, routs, false);
      }
      // masked sums: next registers, then this level's result term
      std::map<int, std::vector<std::pair<size_t, size_t>>> into;   // register -> (step, term)
      std::vector<std::pair<size_t, size_t>> fins;
      for (size_t s : kv.second) {
        const R2Step& st = pr.steps[s];
        for (size_t t = 0; t < st.keep.size(); ++t) into[st.keep[t].dst].push_back({s, t});
        for (size_t t = 0; t < st.fin.size(); ++t) fins.push_back({s, t});
      }
      if (!into.empty()) {
        std::vector<std::vector<MacTerm>> grp;
        std::vector<uint64_t*> go;
        for (int g = 0; g < np; ++g)
          for (auto& kv3 : into) {
            std::vector<MacTerm> terms;
            for (auto& st_t : kv3.second) {
              const R2Step& st = pr.steps[st_t.first];
              const R2Term& tm = st.keep[st_t.second];
              terms.push_back(MacTerm{rot(g, st.src, tm.m), mask(g, first[st_t.first] + st_t.second)});
            }
            grp.push_back(std::move(terms));
            go.push_back(reg(g, kv3.first));
          }
        group_mac(c, level, grp, go, false);
        for (auto& kv3 : into) written[d].push_back(kv3.first);
      }
      if (!fins.empty()) {
        std::vector<std::vector<MacTerm>> grp(np);
        std::vector<uint64_t*> go(np);
        for (int g = 0; g < np; ++g) {
          for (auto& st_t : fins) {
            const R2Step& st = pr.steps[st_t.first];
            const R2Term& tm = st.fin[st_t.second];
            grp[g].push_back(MacTerm{rot(g, st.src, tm.m), mask(g, first[st_t.first] + st.keep.size() + st_t.second)});
          }
          go[g] = oterm(g, d);
        }
        group_mac(c, level, grp, go, true);
      }
    }
    for (auto& kv : written) {
      std::vector<uint64_t*> cts;
      for (int g = 0; g < np; ++g)
        for (int r : kv.second) cts.push_back(reg(g, r));
      rescale_batch(c, la - kv.first, cts);
    }
  }
  std::vector<std::vector<MacTerm>> grp(np);
  for (int d = 0; d < D; ++d) {
    std::vector<uint64_t*> cts(np);
    for (int g = 0; g < np; ++g) cts[g] = oterm(g, d);
    rescale_batch(c, la - d, cts);
    for (int g = 0; g < np; ++g) grp[g].push_back(MacTerm{oterm(g, d), nullptr, la - d});
  }
  group_mac(c, lo, grp, outs, false);
}

// SpIntra-CA of every packed ciphertext Y[g] into outs[g] (batched form)
static void aggregate_batched(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, const std::vector<uint64_t*>& Y,
                              const std::vector<uint64_t*>& outs) {
  const size_t N = c->N;
  const int lv = lp.level_agg, l1 = lv + 1;
  const size_t ct_words = (size_t)2 * l1 * N;
  const size_t ns = lp.shifts.size();
  const int np = (int)Y.size();
  if (lp.family == 3) {
    aggregate_r2_batched(c, ek, lp, Y, outs);
    return;
  }
  auto mask = [&](int g, size_t si) { return (const uint64_t*)lp.ops[(size_t)g * ns + si]; };
  std::vector<const uint64_t*> ysrc(np);
  for (int g = 0; g < np; ++g) ysrc[g] = Y[g] + (size_t)l1 * N;
  if (lp.family == 4) {
    // out_g = Y_g (.) mask_0 + ModDown(sum_delta KeyInner_delta (.) mask_delta) + sum_delta sigma(c0) (.) mask_delta:
    // every rotation of Y_g on its one ModUp, one ModDown per packed ciphertext
    std::vector<std::vector<MacTerm>> init(np);
    std::vector<KSJob> jobs;
    for (int g = 0; g < np; ++g)
      for (size_t si = 0; si < ns; ++si) {
        uint64_t gal;
        const uint64_t* key = rot_key(c, ek, lp.shifts[si], gal);
        if (!key)
          init[g].push_back(MacTerm{Y[g], mask(g, si)});
        else
          jobs.push_back(KSJob{key, Y[g], nullptr, mask(g, si), gal, g, g});
      }
    group_mac(c, lv, init, outs, false);
    keyswitch_masked_sum(c, lv, ysrc, jobs, outs, true);
    rescale_batch(c, lv, outs);
    return;
  }
  if (lp.family == 1) {
    // out_g = sum_delta Rot_delta(Y_g) (.) mask_delta: identity terms first,
    // every rotation (hoisted on Y_g's ModUp) accumulated in the final ModDown step
    std::vector<std::vector<MacTerm>> init(np);
    std::vector<KSJob> jobs;
    for (int g = 0; g < np; ++g)
      for (size_t si = 0; si < ns; ++si) {
        uint64_t gal;
        const uint64_t* key = rot_key(c, ek, lp.shifts[si], gal);
        if (!key)
          init[g].push_back(MacTerm{Y[g], mask(g, si)});
        else
          jobs.push_back(KSJob{key, Y[g], nullptr, mask(g, si), gal, g, g});
      }
    group_mac(c, lv, init, outs, false);
    keyswitch_batch(c, lv, ysrc, jobs, outs, true);
  } else {
    // baby-step giant-step: Rot_{gi G}( sum_b Rot_b(Y_g) (.) mask'_{gi,b} )
    const int64_t G = lp.G;
    std::set<int64_t> babies;
    std::map<int64_t, std::vector<size_t>> giants;
    for (size_t si = 0; si < ns; ++si) {
      const int64_t d = lp.shifts[si];
      if (fmodp(d, G)) babies.insert(fmodp(d, G));
      giants[fdiv(d, G)].push_back(si);
    }
    const int nb = (int)babies.size();
    std::map<int64_t, int> bpos;
    for (int64_t b : babies) bpos.emplace(b, (int)bpos.size());
    // baby rotations of every packed ciphertext, hoisted on its ModUp
    uint64_t* bb = (uint64_t*)dev_scratch(c, 70, std::max<size_t>(1, (size_t)np * nb) * ct_words * 8);
    auto baby = [&](int g, int64_t b) { return bb + ((size_t)g * nb + bpos.at(b)) * ct_words; };
    {
      // key-major: the rotations of every packed ciphertext by one baby step are adjacent, so the
      // batch reads that step's key once for all of them
      std::vector<KSJob> jobs;
      std::vector<uint64_t*> bouts;
      for (int64_t b : babies)
        for (int g = 0; g < np; ++g) {
          uint64_t gal;
          const uint64_t* key = rot_key(c, ek, b, gal);
          if (!key) {
            copy_d2d(c, baby(g, b), Y[g], ct_words * 8);
            continue;
          }
          jobs.push_back(KSJob{key, Y[g], nullptr, nullptr, gal, g, (int)bouts.size()});
          bouts.push_back(baby(g, b));
        }
      keyswitch_batch(c, lv, ysrc, jobs, bouts, false);
    }
    // inner sums: giant 0 straight into the output, the others into buffers
    int n_inner = 0;
    for (auto& kv : giants) n_inner += kv.first != 0;
    uint64_t* ib = (uint64_t*)dev_scratch(c, 71, std::max<size_t>(1, (size_t)np * n_inner) * ct_words * 8);
    std::vector<std::vector<MacTerm>> groups;
    std::vector<uint64_t*> gouts;
    std::vector<const uint64_t*> isrc;
    std::vector<std::vector<MacTerm>> ident(np);
    std::vector<KSJob> jobs;
    if (!giants.count(0))
      for (int g = 0; g < np; ++g) {
        groups.emplace_back();   // an empty group clears the output
        gouts.push_back(outs[g]);
      }
    // giant-major: the groups of one giant step (one per packed ciphertext) are launched
    // next to each other, so its masks, shared by the packed ciphertexts, come from L2
    for (auto& kv : giants) {
      for (int g = 0; g < np; ++g) {
        std::vector<MacTerm> terms;
        for (size_t si : kv.second) {
          const int64_t b = fmodp(lp.shifts[si], G);
          terms.push_back(MacTerm{b ? baby(g, b) : Y[g], mask(g, si)});
        }
        if (kv.first == 0) {
          groups.push_back(terms);
          gouts.push_back(outs[g]);
          continue;
        }
        uint64_t* inner = ib + isrc.size() * ct_words;
        groups.push_back(terms);
        gouts.push_back(inner);
        uint64_t gal;
        const uint64_t* key = rot_key(c, ek, kv.first * G, gal);
        if (!key) {
          ident[g].push_back(MacTerm{inner, nullptr});
        } else {
          jobs.push_back(KSJob{key, inner, nullptr, nullptr, gal, (int)isrc.size(), g});
        }
        isrc.push_back(inner + (size_t)l1 * N);
      }
    }
    std::stable_sort(jobs.begin(), jobs.end(), [](const KSJob& x, const KSJob& y) { return x.grp < y.grp; });
    // packed ciphertexts with the same column count share their masks (one plaintext per
    // shift): then a thread reads each mask word once for up to four of them
    bool shared = c->N >= 512;
    for (int g = 1; g < np && shared; ++g) shared = mask(g, 0) == mask(0, 0);
    if (shared) {
      for (int c0 = 0; c0 < np; c0 += MacTermNP::MAX) {
        const int nc = std::min((int)MacTermNP::MAX, np - c0);
        std::vector<std::vector<MacTermNP>> mg;
        std::vector<uint64_t*> mo;
        for (size_t gi = 0; gi < groups.size(); ++gi) {
          const int g = (int)(gi % np);   // groups go giant-major, packed ciphertext fastest
          if (g != c0) continue;
          std::vector<MacTermNP> terms;
          for (const MacTerm& tm : groups[gi]) {
            MacTermNP t{};
            t.pt = tm.pt;
            terms.push_back(t);
          }
          for (int k = 0; k < nc; ++k) {
            const std::vector<MacTerm>& src = groups[gi + k];
            for (size_t u = 0; u < src.size(); ++u) terms[u].ct[k] = src[u].ct;
            mo.push_back(gouts[gi + k]);
          }
          mg.push_back(terms);
        }
        group_mac_np(c, lv, nc, mg, mo, false);
      }
    } else {
      group_mac(c, lv, groups, gouts, false);
    }
    // giant rotations of each output summed on the key basis, one ModDown per output
    if (!jobs.empty()) keyswitch_masked_sum(c, lv, isrc, jobs, outs, true);
    group_mac(c, lv, ident, outs, true);
  }
  rescale_batch(c, lv, outs);
}

// Layer outputs squared and relinearised (batched form): out_i = Relin(pre_i (x) pre_i)
static void activation_batched(ckks_ctx* c, const ckks_keys* ek, int lo, const std::vector<uint64_t*>& pre,
                               uint64_t* const* out) {
  const size_t N = c->N, l1 = lo + 1;
  const size_t n = pre.size();
  uint64_t* d = (uint64_t*)dev_scratch(c, 48, n * 3 * l1 * N * 8);
  std::vector<TensorJob> tj(n);
  std::vector<const uint64_t*> srcs(n);
  std::vector<KSJob> jobs(n);
  std::vector<uint64_t*> outs(out, out + n);
  for (size_t i = 0; i < n; ++i) {
    uint64_t* di = d + i * 3 * l1 * N;
    tj[i] = TensorJob{pre[i], pre[i], di};
    srcs[i] = di + 2 * l1 * N;
    jobs[i] = KSJob{ek->swk.at(0), di, di + l1 * N, nullptr, 1, (int)i, (int)i};
  }
  tensor_batch(c, lo, tj);
  keyswitch_batch(c, lo, srcs, jobs, outs, false);
}

static void run_layer_eager(ckks_ctx* c, const ckks_keys* ek, ficgcn_plan* p, int li, const uint64_t* const* in,
                            size_t n_in, uint64_t* const* out, size_t n_out, int mode);

// Graph form: the first call for a set of buffers runs the batched form
// eagerly while recording its device tables and scratch, then captures the
// same launch sequence (recorded buffers, no uploads, no host waits) into a
// HIP graph; later calls with the same buffers and keys replay the graph.
static void run_layer_graph(ckks_ctx* c, const ckks_keys* ek, ficgcn_plan* p, int li, const uint64_t* const* in,
                            size_t n_in, uint64_t* const* out, size_t n_out) {
  if (p->graphs.size() < p->layers.size()) p->graphs.resize(p->layers.size());
  auto& g = p->graphs[li];
  // rearranged inputs (no input ciphertexts) are keyed by their buffer
  const std::vector<const uint64_t*> vin =
      in ? std::vector<const uint64_t*>(in, in + n_in) : std::vector<const uint64_t*>{p->layers[li].packed_in};
  const std::vector<uint64_t*> vout(out, out + n_out);
  if (g && !g->failed && g->exec && g->in == vin && g->out == vout && g->keys == ek && g->ctx == c) {
    HIPCHECK(hipGraphLaunch(g->exec, c->stream));
    return;
  }
  if (g && g->failed && g->in == vin && g->out == vout && g->keys == ek && g->ctx == c) {
    run_layer_eager(c, ek, p, li, in, n_in, out, n_out, 1);
    return;
  }
  HIPCHECK(hipStreamSynchronize(c->stream));
  g.reset(new LayerGraph());
  g->in = vin;
  g->out = vout;
  g->keys = ek;
  g->ctx = c;
  // 1. eager run, recording every table and scratch buffer in call order
  g->rec.mode = Recorder::RECORD;
  c->rec = &g->rec;
  try {
    run_layer_eager(c, ek, p, li, in, n_in, out, n_out, 1);
  } catch (...) {
    c->rec = nullptr;
    g.reset();
    throw;
  }
  c->rec = nullptr;
  HIPCHECK(hipStreamSynchronize(c->stream));
  // 2. capture the same sequence on a stream of its own (the context's may be the null stream)
  hipStream_t cap = nullptr, saved = c->stream;
  HIPCHECK(hipStreamCreate(&cap));
  g->rec.mode = Recorder::REPLAY;
  g->rec.cursor = 0;
  c->rec = &g->rec;
  c->stream = cap;
  bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    try {
      run_layer_eager(c, ek, p, li, in, n_in, out, n_out, 1);
    } catch (...) {
      ok = false;
    }
    hipGraph_t graph = nullptr;
    ok = (hipStreamEndCapture(cap, &graph) == hipSuccess) && ok && graph;
    if (ok) {
      g->graph = graph;
      ok = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess;
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
    ok = ok && g->rec.cursor == g->rec.bufs.size();
  }
  c->stream = saved;
  c->rec = nullptr;
  (void)hipGetLastError();
  (void)hipStreamDestroy(cap);
  if (!ok) g->failed = true;
}

void run_layer(ckks_ctx* c, const ckks_keys* ek, ficgcn_plan* p, int li, const uint64_t* const* in, size_t n_in,
               uint64_t* const* out, size_t n_out, int mode) {
  if (mode == 2) {
    LayerPlan& lp = p->layers[li];
    const bool packed = in == nullptr && n_in == 0;
    if (packed && (lp.kind != 0 || !lp.packed_in))
      FICGCN_THROW(EPLAN_, "no input ciphertexts: needs an Inter-CA layer with rearranged inputs");
    if ((!packed && (int)n_in != lp.n_in_cts()) || (int)n_out != lp.n_packed())
      FICGCN_THROW(EPLAN_, "wrong ciphertext count");
    run_layer_graph(c, ek, p, li, in, n_in, out, n_out);
    return;
  }
  run_layer_eager(c, ek, p, li, in, n_in, out, n_out, mode);
}

// Case-1 Inter-CA layer (Sec. 3.2, App. B): acc = sum_i in_i (.) P_i (P_i = A_hat_k (x) W-slice
// of input ciphertext i), rescale, then acc += Rot(acc, step) for each fold step, so the first
// column group's blocks hold sum over every input column
static void inter_rep(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, const uint64_t* const* in, size_t n_in,
                      uint64_t* out, int mode) {
  const size_t N = c->N;
  const int lv = lp.level_in, l1 = lv + 1, lo = lv - 1;
  const size_t lo_words = (size_t)2 * (lo + 1) * N;
  for (int64_t step : lp.fold_steps) {
    uint64_t gal;
    if (!rot_key(c, ek, step, gal)) FICGCN_THROW(EPLAN_, "identity fold step");
  }
  if (mode == 1) {
    std::vector<std::vector<MacTerm>> grp(1);
    for (size_t i = 0; i < n_in; ++i) grp[0].push_back(MacTerm{in[i], lp.ops[i]});
    group_mac(c, lv, grp, {out}, false);
    rescale_batch(c, lv, {out});
    if (lp.fold_steps.empty()) return;
    uint64_t* tmp = (uint64_t*)dev_scratch(c, 38, lo_words * 8);
    for (int64_t step : lp.fold_steps) {
      uint64_t gal;
      const uint64_t* key = rot_key(c, ek, step, gal);
      keyswitch_batch(c, lo, {out + (size_t)(lo + 1) * N}, {KSJob{key, out, nullptr, nullptr, gal, 0, 0}}, {tmp},
                      false);
      group_mac(c, lo, {{MacTerm{tmp, nullptr}}}, {out}, true);
    }
    return;
  }
  zero_fill(c, out, (size_t)2 * l1 * N);
  for (size_t i0 = 0; i0 < n_in; i0 += PtrList::MAX) {
    PtrList a{}, b{};
    const int nk = (int)std::min<size_t>(PtrList::MAX, n_in - i0);
    for (int k = 0; k < nk; ++k) {
      a.p[k] = in[i0 + k];
      b.p[k] = lp.ops[i0 + k];
    }
    pmul_acc(c, out, a, b, nk, l1);
  }
  rescale_inplace(c, out, lv);
  uint64_t* rt = (uint64_t*)c->buf(37, lo_words * 8);
  for (int64_t step : lp.fold_steps) {
    rotate_one(c, ek, out, lo, step, rt);
    add_inplace(c, out, rt, lo + 1, 2);
  }
}

// Block-rotation combination of an input packed in blocks of B: y = sum_s Rot_{sB}(h) (.) cm_s,
// the nonzero offsets' mask products on the key basis before one ModDown.  No rescale.
static void comb_diag(ckks_ctx* c, const ckks_keys* ek, LayerPlan& lp, const uint64_t* h, uint64_t* y, int mode) {
  const size_t N = c->N;
  const int lv = lp.level_in, l1 = lv + 1;
  const size_t na = lp.n_agg_ops();
  std::vector<int64_t> steps;
  std::vector<const uint64_t*> masks;
  for (size_t k = 0; k < lp.comb_shifts.size(); ++k) {
    steps.push_back(lp.comb_shifts[k] * lp.B);
    masks.push_back(lp.ops[na + k]);
  }
  if (mode != 1) {
    masked_sum_plain(c, ek, h, lv, steps, masks, y);
    return;
  }
  std::vector<std::vector<MacTerm>> init(1);
  std::vector<KSJob> jobs;
  for (size_t k = 0; k < steps.size(); ++k) {
    uint64_t gal;
    const uint64_t* key = rot_key(c, ek, steps[k], gal);
    if (!key)
      init[0].push_back(MacTerm{h, masks[k]});
    else
      jobs.push_back(KSJob{key, h, nullptr, masks[k], gal, 0, 0});
  }
  group_mac(c, lv, init, {y}, false);
  if (!jobs.empty()) keyswitch_masked_sum(c, lv, {h + (size_t)l1 * N}, jobs, {y}, true);
}

static void run_layer_eager(ckks_ctx* c, const ckks_keys* ek, ficgcn_plan* p, int li, const uint64_t* const* in,
                            size_t n_in, uint64_t* const* out, size_t n_out, int mode) {
  LayerPlan& lp = p->layers[li];
  const size_t N = c->N;
  const bool packed = in == nullptr && n_in == 0;   // the layer's rearranged inputs
  if (packed && (lp.kind != 0 || mode != 1 || !lp.packed_in))
    FICGCN_THROW(EPLAN_, "no input ciphertexts: needs an Inter-CA layer with rearranged inputs, batched form");
  if (!packed && (int)n_in != lp.n_in_cts()) FICGCN_THROW(EPLAN_, "wrong number of input ciphertexts");
  if ((int)n_out != lp.n_packed()) FICGCN_THROW(EPLAN_, "wrong number of output ciphertexts");
  for (size_t i = 0; i < n_in && in; ++i)
    if (!in[i]) FICGCN_THROW(EINVAL_, "null input ciphertext");
  for (size_t i = 0; i < n_out; ++i)
    if (!out[i]) FICGCN_THROW(EINVAL_, "null output ciphertext");
  for (size_t i = 0; i < lp.ops.size(); ++i)
    if (!lp.ops[i] && lp.op_alias[i] >= 0) lp.ops[i] = lp.ops[lp.op_alias[i]];
  for (uint64_t* o : lp.ops)
    if (!o) FICGCN_THROW(EPLAN_, "plan operands not encoded or loaded");
  ensure_weights(c, lp);
  const int lv = lp.level_in, l1 = lv + 1;
  const size_t ct_words = (size_t)2 * l1 * N;
  if (lp.act && !ek->swk.count(0)) FICGCN_THROW(ENOKEY_, "missing relinearisation key");
  // layer result before the activation goes to `pre` (the outputs when no activation)
  std::vector<uint64_t*> pre(n_out);
  uint64_t* pre_block = nullptr;
  if (lp.act) {
    pre_block = (uint64_t*)dev_scratch(c, 47, n_out * ct_words * 8);
    for (size_t i = 0; i < n_out; ++i) pre[i] = pre_block + i * ct_words;
  } else {
    for (size_t i = 0; i < n_out; ++i) pre[i] = out[i];
  }
  if (lp.kind == 0 && lp.pack) {
    if (packed) FICGCN_THROW(EPLAN_, "rearranged inputs are for one column per ciphertext");
    inter_rep(c, ek, lp, in, n_in, pre[0], mode);
  } else if (lp.kind == 1 && lp.comb) {
    uint64_t* y = (uint64_t*)dev_scratch(c, 36, ct_words * 8);
    comb_diag(c, ek, lp, in[0], y, mode);
    int lvc = lv;
    for (int r = 0; r < lp.n_rescale_comb;) {
      if (mode == 1 && r + 2 <= lp.n_rescale_comb) {
        rescale2_batch(c, lvc, {y});
        lvc -= 2;
        r += 2;
        continue;
      }
      if (mode == 1)
        rescale_batch(c, lvc, {y});
      else
        rescale_inplace(c, y, lvc);
      --lvc;
      ++r;
    }
    if (lvc != lp.level_agg) FICGCN_THROW(EPLAN_, "inconsistent schedule");
    if (mode == 1)
      aggregate_batched(c, ek, lp, {y}, pre);
    else
      aggregate(c, ek, lp, 0, y, pre[0]);
  } else if (lp.kind == 0) {
    const int F = lp.f_in, K = lp.K;
    if (mode == 1) {
      if (K > PtrList::MAX) FICGCN_THROW(EPLAN_, "batched form supports at most 16 Inter-CA copies");
      PtrList pts{};
      for (int k = 0; k < K; ++k) pts.p[k] = lp.ops[k];
      if (packed) {
        fused_pass_packed(c, lp, pre, pts, K, "inter_fused");
      } else {
        const uint64_t* base = nullptr;
        size_t stride = 0;
        const uint64_t* const* idv = nullptr;
        if (!strided(in, n_in, ct_words, base, stride)) {
          std::vector<const uint64_t*> ins(in, in + n_in);
          idv = upload_ptrs(c, ins, 31);
          base = nullptr;
        }
        fused_pass(c, lp, pre, base, stride, idv, pts, K, "inter_fused");
      }
    } else {
      const int CH = 64;
      uint64_t* Z = (uint64_t*)c->buf(34, (size_t)CH * ct_words * 8);
      for (int l = 0; l < lp.f_out; ++l) zero_fill(c, pre[l], ct_words);
      for (int f0 = 0; f0 < F; f0 += CH) {
        int nf = std::min(CH, F - f0);
        for (int f = 0; f < nf; ++f) {
          uint64_t* z = Z + (size_t)f * ct_words;
          zero_fill(c, z, ct_words);
          for (int k0 = 0; k0 < K; k0 += PtrList::MAX) {
            PtrList a{}, b{};
            int nk = std::min((int)PtrList::MAX, K - k0);
            for (int k = 0; k < nk; ++k) {
              a.p[k] = in[(size_t)(k0 + k) * F + f0 + f];
              b.p[k] = lp.ops[k0 + k];
            }
            pmul_acc(c, z, a, b, nk, l1);
          }
        }
        for (int l = 0; l < lp.f_out; ++l)
          for (int t0 = 0; t0 < nf; t0 += PtrList::MAX) {
            PtrList a{};
            int nt = std::min((int)PtrList::MAX, nf - t0);
            for (int t = 0; t < nt; ++t) a.p[t] = Z + (size_t)(t0 + t) * ct_words;
            smul_acc(c, pre[l], a, lp.w_dev + (((size_t)l * F + f0 + t0) * l1) * 2, nt, l1);
          }
      }
    }
    if (mode == 1) {
      rescale2_batch(c, lv, pre);
    } else {
      for (int l = 0; l < lp.f_out; ++l) {
        rescale_inplace(c, pre[l], lv);
        rescale_inplace(c, pre[l], lv - 1);
      }
    }
  } else {
    // combination at one column per ciphertext
    const int F = lp.f_in;
    uint64_t* cols = (uint64_t*)dev_scratch(c, 35, (size_t)lp.f_out * ct_words * 8);
    std::vector<uint64_t*> colp(lp.f_out);
    for (int l = 0; l < lp.f_out; ++l) colp[l] = cols + (size_t)l * ct_words;
    if (mode == 1) {
      const uint64_t* base = nullptr;
      size_t stride = 0;
      const uint64_t* const* idv = nullptr;
      if (!strided(in, n_in, ct_words, base, stride)) {
        std::vector<const uint64_t*> ins(in, in + n_in);
        idv = upload_ptrs(c, ins, 31);
        base = nullptr;
      }
      fused_pass(c, lp, colp, base, stride, idv, PtrList{}, 0, "comb_fused");
    } else {
      for (int l = 0; l < lp.f_out; ++l) {
        zero_fill(c, colp[l], ct_words);
        for (int t0 = 0; t0 < F; t0 += PtrList::MAX) {
          PtrList a{};
          int nt = std::min((int)PtrList::MAX, F - t0);
          for (int t = 0; t < nt; ++t) a.p[t] = in[t0 + t];
          smul_acc(c, colp[l], a, lp.w_dev + (((size_t)l * F + t0) * l1) * 2, nt, l1);
        }
      }
    }
    int lvc = lv;
    for (int r = 0; r < lp.n_rescale_comb;) {
      if (mode == 1 && r + 2 <= lp.n_rescale_comb) {
        rescale2_batch(c, lvc, colp);
        lvc -= 2;
        r += 2;
        continue;
      }
      if (mode == 1)
        rescale_batch(c, lvc, colp);
      else
        for (int l = 0; l < lp.f_out; ++l) rescale_inplace(c, colp[l], lvc);
      --lvc;
      ++r;
    }
    if (lvc != lp.level_agg) FICGCN_THROW(EPLAN_, "inconsistent schedule");
    const size_t agg_words = (size_t)2 * (lvc + 1) * N;
    const int np = lp.n_packed();
    if (mode == 1) {
      // pack t columns per ciphertext: Y_g = col_{gt} + sum_l Rot_{-(l mod t) B}(col_l)
      uint64_t* yb = (uint64_t*)dev_scratch(c, 36, (size_t)np * agg_words * 8);
      std::vector<uint64_t*> Y(np);
      std::vector<std::vector<MacTerm>> init(np);
      std::vector<const uint64_t*> srcs;
      std::vector<KSJob> jobs;
      for (int g = 0; g < np; ++g) {
        Y[g] = yb + (size_t)g * agg_words;
        init[g].push_back(MacTerm{colp[(size_t)g * lp.t], nullptr});
        for (int l = g * lp.t + 1; l < std::min(lp.f_out, (g + 1) * lp.t); ++l) {
          uint64_t gal;
          const uint64_t* key = rot_key(c, ek, -(int64_t)(l % lp.t) * lp.B, gal);
          if (!key) {
            init[g].push_back(MacTerm{colp[l], nullptr});
            continue;
          }
          jobs.push_back(KSJob{key, colp[l], nullptr, nullptr, gal, (int)srcs.size(), g});
          srcs.push_back(colp[l] + (size_t)(lvc + 1) * N);
        }
      }
      group_mac(c, lvc, init, Y, false);
      keyswitch_batch(c, lvc, srcs, jobs, Y, true);
      aggregate_batched(c, ek, lp, Y, pre);
    } else {
      uint64_t* y = (uint64_t*)c->buf(36, agg_words * 8);
      uint64_t* rt = (uint64_t*)c->buf(37, agg_words * 8);
      for (int g = 0; g < np; ++g) {
        copy_d2d(c, y, colp[(size_t)g * lp.t], agg_words * 8);
        for (int l = g * lp.t + 1; l < std::min(lp.f_out, (g + 1) * lp.t); ++l) {
          rotate_one(c, ek, colp[l], lvc, -(int64_t)(l % lp.t) * lp.B, rt);
          add_inplace(c, y, rt, lvc + 1, 2);
        }
        aggregate(c, ek, lp, g, y, pre[g]);
      }
    }
  }
  if (lp.act && mode == 1) {
    activation_batched(c, ek, lp.level_out, pre, out);
  } else if (lp.act) {
    const int lo = lp.level_out;
    for (size_t i = 0; i < n_out; ++i) {
      // out = pre^2 with relinearisation at the layer's output level
      const size_t l1o = lo + 1, ext = l1o + c->alpha;
      const int nd = (int)((l1o + c->alpha - 1) / c->alpha);
      uint64_t* d = (uint64_t*)dev_scratch(c, 48, 3 * l1o * N * 8);
      tensor(c, pre[i], pre[i], d, lo);
      uint64_t* D = (uint64_t*)c->buf(40, (size_t)nd * ext * N * 8);
      uint64_t* acc = (uint64_t*)c->buf(41, 2 * ext * N * 8);
      modup(c, d + 2 * l1o * N, lo, D);
      keymac(c, acc, D, ek->swk.at(0), lo, 1);
      moddown(c, acc, lo, out[i], d, 1, d + l1o * N);
    }
  }
}

}  // namespace ficgcn

using namespace ficgcn;

static ficgcn_status plan_guard_status(const Error& e) {
  set_error(e.msg);
  return (ficgcn_status)e.code;
}

#define GUARD_BEGIN try {
#define GUARD_END                                   \
  return FICGCN_OK;                                 \
  }                                                 \
  catch (const Error& e) { return plan_guard_status(e); } \
  catch (const std::exception& e) {                 \
    set_error(e.what());                            \
    return FICGCN_EINVAL;                           \
  }

extern "C" {

ficgcn_status ficgcn_plan_create(ckks_ctx* ctx, const int32_t* rowptr, const int32_t* col, const double* val,
                                 uint32_t n_v, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                                 const ficgcn_plan_opts* opts, ficgcn_plan** out) {
  GUARD_BEGIN
  if (!ctx || !rowptr || !col || !val || !dims || !weights || !opts || !out || n_v == 0 || n_layers == 0)
    FICGCN_THROW(EINVAL_, "null or empty argument");
  if (opts->family < 0 || opts->family > 4) FICGCN_THROW(EINVAL_, "family must be 0, 1, 2, 3 or 4");
  for (uint32_t l = 0; l < n_layers; ++l)
    if (!weights[l] || dims[l] == 0 || dims[l + 1] == 0) FICGCN_THROW(EINVAL_, "bad layer dimensions or weights");
  std::unique_ptr<ficgcn_plan> p(new ficgcn_plan());
  p->ctx = ctx;
  p->n_v = (int)n_v;
  p->rowptr.assign(rowptr, rowptr + n_v + 1);
  if (p->rowptr[0] != 0) FICGCN_THROW(EINVAL_, "rowptr[0] must be 0");
  for (uint32_t v = 0; v < n_v; ++v)
    if (p->rowptr[v + 1] < p->rowptr[v]) FICGCN_THROW(EINVAL_, "rowptr not monotone");
  const int nnz = p->rowptr[n_v];
  p->col.assign(col, col + nnz);
  p->val.assign(val, val + nnz);
  for (uint32_t v = 0; v < n_v; ++v) {
    // rows sorted by column, as the routing and copy order read them
    std::vector<std::pair<int32_t, double>> r;
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e) {
      if (p->col[e] < 0 || p->col[e] >= (int32_t)n_v) FICGCN_THROW(EINVAL_, "column index out of range");
      r.push_back({p->col[e], p->val[e]});
    }
    std::sort(r.begin(), r.end());
    for (size_t i = 0; i + 1 < r.size(); ++i)
      if (r[i].first == r[i + 1].first) FICGCN_THROW(EINVAL_, "duplicate column in a row");
    for (size_t i = 0; i < r.size(); ++i) {
      p->col[p->rowptr[v] + i] = r[i].first;
      p->val[p->rowptr[v] + i] = r[i].second;
    }
  }
  build_plan(ctx, p.get(), dims, n_layers, weights, *opts);
  for (auto& lp : p->layers) lp.ops.assign(plan_operand_count(p.get(), (int)(&lp - &p->layers[0])), nullptr);
  *out = p.release();
  GUARD_END
}

void ficgcn_plan_destroy(ficgcn_plan* plan) { delete plan; }

ficgcn_status ficgcn_plan_node_order(const ficgcn_plan* plan, int32_t* pi_out) {
  GUARD_BEGIN
  if (!plan || !pi_out) FICGCN_THROW(EINVAL_, "null argument");
  std::memcpy(pi_out, plan->pi.data(), plan->pi.size() * 4);
  GUARD_END
}

ficgcn_status ficgcn_plan_copy_sources(const ficgcn_plan* plan, uint32_t layer, int32_t* src_out) {
  GUARD_BEGIN
  if (!plan || !src_out || layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "bad argument");
  const LayerPlan& lp = plan->layers[layer];
  if (lp.kind != 0) FICGCN_THROW(EPLAN_, "not an Inter-CA layer");
  std::memcpy(src_out, lp.copy_src.data(), lp.copy_src.size() * 4);
  GUARD_END
}

ficgcn_status ficgcn_plan_rot_steps(const ficgcn_plan* plan, int64_t* steps_out, size_t cap, size_t* n_out) {
  GUARD_BEGIN
  if (!plan || !n_out) FICGCN_THROW(EINVAL_, "null argument");
  *n_out = plan->rot_steps.size();
  for (size_t i = 0; i < plan->rot_steps.size() && i < cap && steps_out; ++i) steps_out[i] = plan->rot_steps[i];
  GUARD_END
}

ficgcn_status ficgcn_plan_info(const ficgcn_plan* plan, int64_t* info_out, double* scales_out, uint32_t* n_layers) {
  GUARD_BEGIN
  if (!plan || !n_layers) FICGCN_THROW(EINVAL_, "null argument");
  *n_layers = (uint32_t)plan->layers.size();
  for (size_t li = 0; li < plan->layers.size(); ++li) {
    const LayerPlan& lp = plan->layers[li];
    if (info_out) {
      int64_t* o = info_out + li * 18;
      o[0] = lp.kind;
      o[1] = lp.f_in;
      o[2] = lp.f_out;
      o[3] = lp.K;
      o[4] = lp.t;
      o[5] = lp.B;
      o[6] = lp.family;
      o[7] = lp.G;
      o[8] = (int64_t)lp.shifts.size();
      o[9] = lp.level_in;
      o[10] = lp.level_out;
      o[11] = lp.n_in_cts();
      o[12] = lp.n_packed();
      o[13] = lp.pack;
      o[14] = lp.comb;
      o[15] = (int64_t)lp.fold_steps.size();
      o[16] = (int64_t)lp.comb_shifts.size();
      o[17] = lp.paper_mode;
    }
    if (scales_out) {
      scales_out[li * 5] = lp.scale_in;
      scales_out[li * 5 + 1] = lp.scale_out;
      scales_out[li * 5 + 2] = lp.sW;
      scales_out[li * 5 + 3] = lp.mode_cost_inter;
      scales_out[li * 5 + 4] = lp.mode_cost_spintra;
    }
  }
  GUARD_END
}

ficgcn_status ficgcn_plan_shifts(const ficgcn_plan* plan, uint32_t layer, int64_t* out, size_t cap, size_t* n_out) {
  GUARD_BEGIN
  if (!plan || !n_out || layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "bad argument");
  const auto& s = plan->layers[layer].shifts;
  *n_out = s.size();
  for (size_t i = 0; i < s.size() && i < cap && out; ++i) out[i] = s[i];
  GUARD_END
}

ficgcn_status ficgcn_plan_weights_int(const ficgcn_plan* plan, uint32_t layer, int64_t* out) {
  GUARD_BEGIN
  if (!plan || !out || layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "bad argument");
  const auto& w = plan->layers[layer].w_int;
  std::memcpy(out, w.data(), w.size() * 8);
  GUARD_END
}

ficgcn_status ficgcn_plan_operand_count(const ficgcn_plan* plan, uint32_t layer, size_t* n_out) {
  GUARD_BEGIN
  if (!plan || !n_out || layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "bad argument");
  *n_out = plan_operand_count(plan, (int)layer);
  GUARD_END
}

ficgcn_status ficgcn_plan_operand_slots(const ficgcn_plan* plan, uint32_t layer, size_t i, double* slots_out) {
  GUARD_BEGIN
  if (!plan || !slots_out || layer >= plan->layers.size() || i >= plan_operand_count(plan, (int)layer))
    FICGCN_THROW(EINVAL_, "bad argument");
  std::vector<double> v;
  plan_operand_slots(plan, (int)layer, i, v);
  std::memcpy(slots_out, v.data(), v.size() * 8);
  GUARD_END
}

// operands sharing another's memory point where it points once it is set
static void resolve_aliases(LayerPlan& lp) {
  for (size_t i = 0; i < lp.ops.size(); ++i)
    if (lp.op_alias[i] >= 0 && !lp.ops[i]) lp.ops[i] = lp.ops[lp.op_alias[i]];
}

static void ensure_ops_block(ckks_ctx* ctx, LayerPlan& lp) {
  if (lp.ops_block) return;
  if (hipMalloc(&lp.ops_block, std::max<size_t>(1, lp.op_words) * 8) != hipSuccess)
    FICGCN_THROW(ENOMEM_, "operand allocation failed");
}

ficgcn_status ficgcn_plan_operand_level(const ficgcn_plan* plan, uint32_t layer, size_t i, uint32_t* level_out,
                                        double* scale_out) {
  GUARD_BEGIN
  if (!plan || !level_out || layer >= plan->layers.size() || i >= plan_operand_count(plan, (int)layer))
    FICGCN_THROW(EINVAL_, "bad argument");
  *level_out = (uint32_t)plan_operand_level(plan, (int)layer, i);
  if (scale_out) *scale_out = plan_operand_scale(plan, (int)layer, i);
  GUARD_END
}

ficgcn_status ficgcn_plan_radix2_stats(const ficgcn_plan* plan, uint32_t layer, int64_t* out) {
  GUARD_BEGIN
  if (!plan || !out || layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "bad argument");
  const LayerPlan& lp = plan->layers[layer];
  if (lp.kind != 1 || lp.family != 3) FICGCN_THROW(EPLAN_, "not a radix-2 SpIntra-CA layer");
  const R2Program& r = lp.r2;
  std::set<std::pair<int, int64_t>> rots;
  std::set<int64_t> amounts;
  for (const R2Step& st : r.steps) {
    for (const auto* v : {&st.keep, &st.fin})
      for (const R2Term& t : *v)
        if (t.m) {
          rots.insert({st.src, t.m});
          amounts.insert(t.m);
        }
  }
  out[0] = r.n_lanes;
  out[1] = (int64_t)r.steps.size();
  out[2] = (int64_t)rots.size();
  out[3] = (int64_t)amounts.size();
  out[4] = r.depth;
  out[5] = (int64_t)r.ops.size();
  out[6] = r.n_moved;
  out[7] = (int64_t)r.reg_depth.size() - 1;
  GUARD_END
}

ficgcn_status ficgcn_plan_encode(ckks_ctx* ctx, ficgcn_plan* plan) {
  GUARD_BEGIN
  if (!ctx || !plan) FICGCN_THROW(EINVAL_, "null argument");
  ensure_device(ctx);
  for (size_t li = 0; li < plan->layers.size(); ++li) {
    LayerPlan& lp = plan->layers[li];
    ensure_ops_block(ctx, lp);
    const size_t n = lp.ops.size();
    const size_t chunk = 256;
    std::vector<double> all;
    std::vector<double> v;
    // runs of operands with one level, basis and scale; operands sharing another's memory
    // (op_alias) are that operand
    for (size_t b0 = 0; b0 < n;) {
      if (lp.op_alias[b0] >= 0) {
        ++b0;
        continue;
      }
      size_t nb = 1;
      const double sc = plan_operand_scale(plan, (int)li, b0);
      while (b0 + nb < n && nb < chunk && lp.op_alias[b0 + nb] < 0 && lp.op_lv[b0 + nb] == lp.op_lv[b0] &&
             lp.op_x[b0 + nb] == lp.op_x[b0] && plan_operand_scale(plan, (int)li, b0 + nb) == sc)
        ++nb;
      all.assign(nb * plan->M, 0.0);
      for (size_t b = 0; b < nb; ++b) {
        plan_operand_slots(plan, (int)li, b0 + b, v);
        std::memcpy(all.data() + b * plan->M, v.data(), plan->M * 8);
      }
      if (lp.op_x[b0]) {
        encode_batch_ext(ctx, all.data(), nb, plan->M, sc, lp.op_lv[b0], lp.ops_block + lp.op_off[b0]);
      } else {
        ficgcn_status st = ckks_encode_batch(ctx, all.data(), nb, plan->M, sc, lp.op_lv[b0],
                                             lp.ops_block + lp.op_off[b0]);
        if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
      }
      for (size_t b = 0; b < nb; ++b) lp.ops[b0 + b] = lp.ops_block + lp.op_off[b0 + b];
      b0 += nb;
    }
    resolve_aliases(lp);
  }
  GUARD_END
}

ficgcn_status ficgcn_plan_load_operand(ckks_ctx* ctx, ficgcn_plan* plan, uint32_t layer, size_t i,
                                       const uint64_t* host_coeffs) {
  GUARD_BEGIN
  if (!ctx || !plan || !host_coeffs || layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "bad argument");
  ensure_device(ctx);
  LayerPlan& lp = plan->layers[layer];
  if (i >= lp.ops.size()) FICGCN_THROW(EINVAL_, "operand index out of range");
  ensure_ops_block(ctx, lp);
  uint64_t* dst = lp.ops_block + lp.op_off[i];
  if (lp.op_x[i]) {
    pt_load_ext(ctx, host_coeffs, lp.op_lv[i], dst);
  } else {
    ficgcn_status st = ckks_pt_load(ctx, host_coeffs, lp.op_lv[i], dst);
    if (st != FICGCN_OK) FICGCN_THROW(st, ficgcn_last_error());
  }
  lp.ops[i] = dst;
  GUARD_END
}

ficgcn_status ficgcn_plan_fill_operands(ckks_ctx* ctx, ficgcn_plan* plan, uint64_t seed) {
  GUARD_BEGIN
  if (!ctx || !plan) FICGCN_THROW(EINVAL_, "null argument");
  ensure_device(ctx);
  for (size_t li = 0; li < plan->layers.size(); ++li) {
    LayerPlan& lp = plan->layers[li];
    ensure_ops_block(ctx, lp);
    for (size_t i = 0; i < lp.ops.size(); ++i) {
      if (lp.op_alias[i] >= 0) continue;
      uint64_t* dst = lp.ops_block + lp.op_off[i];
      const int l1 = lp.op_lv[i] + 1;
      // stream (6, layer * 2^20 + i, limb): a stream the scheme itself never draws
      sample_uniform(ctx, dst, seed, 6, (uint32_t)(li << 20 | i), 0, l1 + (lp.op_x[i] ? ctx->alpha : 0),
                     lp.op_x[i] ? lm_ext(lp.op_lv[i], ctx->L) : lm_q(l1), 1);
      lp.ops[i] = dst;
    }
    resolve_aliases(lp);
  }
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  GUARD_END
}

ficgcn_status ficgcn_plan_packed_input_words(const ficgcn_plan* plan, ckks_ctx* ctx, uint32_t layer,
                                             uint64_t* words_out) {
  GUARD_BEGIN
  if (!ctx || !plan || !words_out) FICGCN_THROW(EINVAL_, "null argument");
  if (layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "layer index out of range");
  const LayerPlan& lp = plan->layers[layer];
  if (lp.kind != 0) FICGCN_THROW(EPLAN_, "only an Inter-CA layer's inputs are rearranged");
  if (!mfma_pack_supported(ctx)) FICGCN_THROW(EPLAN_, "rearranged inputs need primes below 2^51");
  *words_out = mfma_packed_words(ctx, lp.K, lp.f_in, lp.level_in);
  GUARD_END
}

ficgcn_status ficgcn_plan_pack_inputs(ckks_ctx* ctx, ficgcn_plan* plan, uint32_t layer, const uint64_t* const* in_cts,
                                      size_t n_in, uint64_t* packed_dev, uint64_t packed_words) {
  GUARD_BEGIN
  if (!ctx || !plan || !in_cts || !packed_dev) FICGCN_THROW(EINVAL_, "null argument");
  if (layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "layer index out of range");
  LayerPlan& lp = plan->layers[layer];
  if (lp.kind != 0) FICGCN_THROW(EPLAN_, "only an Inter-CA layer's inputs are rearranged");
  if ((int)n_in != lp.n_in_cts()) FICGCN_THROW(EPLAN_, "wrong number of input ciphertexts");
  for (size_t i = 0; i < n_in; ++i)
    if (!in_cts[i]) FICGCN_THROW(EINVAL_, "null input ciphertext");
  ensure_device(ctx);
  ensure_weights(ctx, lp);
  if (lp.K > PtrList::MAX || !ensure_mfma_weights(ctx, lp, lp.K))
    FICGCN_THROW(EPLAN_, "layer shape or weights outside the matrix-core pass");
  if (packed_words < mfma_packed_words(ctx, lp.K, lp.f_in, lp.level_in)) FICGCN_THROW(EINVAL_, "buffer too small");
  const size_t ct_words = (size_t)2 * (lp.level_in + 1) * ctx->N;
  const uint64_t* base = nullptr;
  size_t stride = 0;
  const uint64_t* const* idv = nullptr;
  if (!strided(in_cts, n_in, ct_words, base, stride)) {
    std::vector<const uint64_t*> ins(in_cts, in_cts + n_in);
    idv = upload_ptrs(ctx, ins, 31);
    base = nullptr;
  }
  mfma_pack(ctx, base, stride, idv, lp.K, lp.f_in, lp.level_in, packed_dev);
  HIPCHECK(hipStreamSynchronize(ctx->stream));
  lp.packed_in = packed_dev;
  GUARD_END
}

ficgcn_status ficgcn_gcn_layer(ckks_ctx* ctx, const ckks_keys* eval_keys, const ficgcn_plan* plan, uint32_t layer,
                               const uint64_t* const* in_cts, size_t n_in, uint64_t* const* out_cts, size_t n_out,
                               int32_t mode) {
  GUARD_BEGIN
  if (!ctx || !eval_keys || !plan || (!in_cts && n_in) || !out_cts) FICGCN_THROW(EINVAL_, "null argument");
  if (layer >= plan->layers.size()) FICGCN_THROW(EINVAL_, "layer index out of range");
  if (mode < 0 || mode > 2) FICGCN_THROW(EINVAL_, "mode must be 0 (plain), 1 (batched) or 2 (batched, graph)");
  ensure_device(ctx);
  run_layer(ctx, eval_keys, const_cast<ficgcn_plan*>(plan), (int)layer, in_cts, n_in, out_cts, n_out, mode);
  GUARD_END
}

}  // extern "C"
