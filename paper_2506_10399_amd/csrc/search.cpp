// Plan search: candidate enumeration, local-adjacency features, the analytic
// judge (algorithmic bytes of a plan's batched execution) and the
// model-pruned search.
//
// Candidates vary what the paper's planner decides for a SpIntra-CA layer:
// the packing t (Sec. 3.2, App. B), the node order (NOO of Sec. 3.4 on or off,
// and its region cap TH) and the routing family.  The judge builds a
// candidate's plan and counts the HBM bytes each operation of the batched
// form must move; a learned model predicts latency from features that need
// no plan, so only its best few candidates are built.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <set>

#include "../../include/ficgcn.h"
#include "plan.h"

namespace ficgcn {

void mlp_predict(ficgcn_mlp* a, const float* x_dev, size_t rows, float* y_dev);

static int next_pow2i(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

static int ilog2(int x) {
  int l = 0;
  while ((1 << (l + 1)) <= x) ++l;
  return l;
}

// largest feasible packing t (1 when no layer is SpIntra-CA)
static int t_max_of(uint32_t n_v, const uint32_t* dims, uint32_t n_layers, int M, int first_mode) {
  int t = 0;
  for (uint32_t i = 0; i < n_layers; ++i)
    if (i > 0 || first_mode == 1) {
      if (i + 1 < n_layers) return 1;   // a SpIntra-CA layer feeding another keeps one column per ciphertext
      t = t == 0 ? next_pow2i((int)dims[i + 1]) : std::min(t, next_pow2i((int)dims[i + 1]));
    }
  if (t == 0) return 1;
  return std::min(t, M / next_pow2i((int)n_v));
}

static std::vector<ficgcn_plan_opts> candidates(uint32_t n_v, const uint32_t* dims, uint32_t n_layers, uint32_t log_n,
                                                const ficgcn_plan_opts& base) {
  const int M = 1 << (log_n - 1);
  std::vector<ficgcn_plan_opts> out;
  bool spintra = base.first_mode == 1 || n_layers > 1;
  if (!spintra) {
    out.push_back(base);
    return out;
  }
  const int tmax = t_max_of(n_v, dims, n_layers, M, base.first_mode);
  std::vector<int> ths;
  for (int th : {64, 256, 1024, 4096})
    if (th < (int)n_v) ths.push_back(th);
  ths.push_back((int)n_v);
  for (int t = 1; t <= tmax; t <<= 1) {
    const int B = M / t;
    for (int noo = 0; noo < 2; ++noo) {
      if (!noo && (int)n_v > B) continue;
      const std::vector<int> th_list = noo ? ths : std::vector<int>{0};
      for (int th : th_list)
        for (int fam : {1, 2, 4}) {
          ficgcn_plan_opts o = base;
          o.t = t;
          o.use_noo = noo;
          o.TH = noo ? th : 0;
          o.family = fam;
          out.push_back(o);
        }
    }
  }
  return out;
}

// shift count and baby+giant count of the identity order at block size B
static void identity_shifts(const int32_t* rowptr, const int32_t* col, uint32_t n_v, int M, int B, double& n_shift,
                            double& n_bsgs) {
  const bool wrap = B == M;
  std::set<int64_t> sh;
  for (uint32_t v = 0; v < n_v; ++v)
    for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      int64_t d = (int64_t)col[e] - (int64_t)v;
      if (wrap) {
        d %= M;
        if (d > M / 2) d -= M;
        if (d <= -M / 2) d += M;
      }
      sh.insert(d);
    }
  n_shift = (double)sh.size();
  // babies + giants of the best power-of-two split
  double best = n_shift;
  for (int G = 2; G <= B; G <<= 1) {
    std::set<int64_t> b, g;
    for (int64_t d : sh) {
      int64_t q = d >= 0 ? d / G : -((-d + G - 1) / G);
      int64_t r = d - q * G;
      if (r) b.insert(r);
      if (q) g.insert(q);
    }
    best = std::min(best, (double)(b.size() + g.size()));
  }
  n_bsgs = best;
}

static void features(const int32_t* rowptr, const int32_t* col, uint32_t n_v, const uint32_t* dims,
                     uint32_t n_layers, uint32_t log_n, const ficgcn_plan_opts& o, float* out) {
  const int M = 1 << (log_n - 1);
  const int nnz = rowptr[n_v];
  // degree statistics (off-diagonal entries of each row)
  double dsum = 0, d2 = 0, dmax = 0;
  double loc_sum = 0, near32 = 0, near1k = 0, n_edges = 0;
  for (uint32_t v = 0; v < n_v; ++v) {
    int d = 0;
    for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      if (col[e] == (int32_t)v) continue;
      ++d;
      const double gap = std::fabs((double)col[e] - (double)v);
      loc_sum += std::log2(gap + 1.0);
      near32 += gap < 32;
      near1k += gap < 1024;
      n_edges += 1;
    }
    dsum += d;
    d2 += (double)d * d;
    dmax = std::max(dmax, (double)d);
  }
  const double dmean = dsum / n_v;
  const double dcv = dmean > 0 ? std::sqrt(std::max(0.0, d2 / n_v - dmean * dmean)) / dmean : 0.0;
  const double ne = std::max(1.0, n_edges);
  // the SpIntra-CA layer the candidate shapes (the last layer)
  const int li = (int)n_layers - 1;
  const int f_in = (int)dims[li], f_out = (int)dims[li + 1];
  const int t = std::max(1, o.t);
  const int B = M / t;
  const int TH = o.use_noo ? (o.TH > 0 ? o.TH : ((int)n_v < 10000 ? 1024 : 4096)) : (int)n_v;
  double n_shift, n_bsgs;
  identity_shifts(rowptr, col, n_v, M, B, n_shift, n_bsgs);
  const double n_packed = std::ceil((double)f_out / t);
  float f[FICGCN_N_FEATURES] = {
      (float)std::log2((double)n_v) / 16.0f,
      (float)std::log2((double)std::max(1, nnz)) / 20.0f,
      (float)(dmean / 16.0),
      (float)(std::log2(dmax + 1.0) / 10.0),
      (float)dcv,
      (float)(loc_sum / ne / std::max(1.0, std::log2((double)M))),
      (float)(near32 / ne),
      (float)(near1k / ne),
      (float)(ilog2(t) / 6.0),
      (float)(ilog2(B) / 16.0),
      (float)((double)n_v / B),
      (float)(o.use_noo ? 1 : 0),
      (float)(std::log2((double)std::max(1, TH)) / 16.0),
      (float)(o.family == 1),
      (float)(o.family == 2),
      (float)(o.family == 4),
      (float)(std::log2((double)f_in + 1.0) / 12.0),
      (float)(std::log2((double)f_out + 1.0) / 12.0),
      (float)(std::log2(n_packed + 1.0) / 6.0),
      (float)(std::log2((double)M) / 16.0),
      (float)(std::log2(std::ceil((double)n_v / std::max(1, TH)) + 1.0) / 8.0),
      (float)(std::log2(n_shift + 1.0) / 16.0),
      (float)(std::log2(n_bsgs + 1.0) / 16.0),
      (float)(n_layers / 4.0),
  };
  std::memcpy(out, f, sizeof(f));
}

// HBM bytes of one batched inference of the plan, every pass of the batched
// launch sequence counted (in limbs of N words): an NTT of n limbs moves 4n
// (two passes, read and write); a ModUp at level l (L1 = l + 1 limbs, beta
// digits, ext = L1 + alpha) moves 4 L1 + 5 beta ext (copy, inverse NTT,
// conversion, forward NTT of the converted limbs); a key inner product
// 3 beta ext + 2 ext (digits, key, accumulator); a ModDown with its final
// step 10 alpha + 17 L1; a rescale 14 l + 16; a masked-sum term 3 L1.
static double plan_bytes(const ficgcn_plan* p) {
  const ckks_ctx* c = p->ctx;
  const double limb = 8.0 * c->N;
  const int a = c->alpha;
  auto beta = [&](int L1) { return (double)((L1 + a - 1) / a); };
  auto modup = [&](int l) {
    const double L1 = l + 1, ext = L1 + a;
    return limb * (4.0 * L1 + 5.0 * beta(l + 1) * ext);
  };
  auto inner = [&](int l) {
    const double ext = l + 1 + a;
    return limb * (3.0 * beta(l + 1) * ext + 2.0 * ext);
  };
  auto moddown = [&](int l) { return limb * (10.0 * a + 17.0 * (l + 1)); };
  auto ks_single = [&](int l) { return modup(l) + inner(l) + moddown(l); };
  auto ks_extra = [&](int l) { return inner(l) + moddown(l); };
  auto mask = [&](int l) { return limb * 3.0 * (l + 1); };
  auto rs = [&](int l) { return limb * (14.0 * l + 16.0); };
  double bytes = 0;
  for (const LayerPlan& lp : p->layers) {
    const int l1 = lp.level_in + 1;
    int n_out_cts;
    if (lp.kind == 0 && lp.pack) {
      // case-1 layout: every input ciphertext and its plaintext once, one output, its rescale,
      // then one switch and one addition per fold rotation
      const int n_in = lp.n_in_cts(), lo = lp.level_in - 1;
      bytes += limb * l1 * (3.0 * n_in + 2.0) + rs(lp.level_in);
      bytes += lp.fold_steps.size() * (ks_single(lo) + limb * 6.0 * (lo + 1));
      n_out_cts = 1;
    } else if (lp.kind == 0) {
      bytes += limb * l1 * (2.0 * lp.K * lp.f_in + lp.K + 2.0 * lp.f_out) + 8.0 * l1 * lp.f_in * lp.f_out;
      bytes += lp.f_out * (rs(lp.level_in) + rs(lp.level_in - 1));
      n_out_cts = lp.f_out;
    } else {
      const int la = lp.level_agg;
      const int np = lp.n_packed();
      if (lp.comb) {
        // block-rotation combination: one ModUp, per nonzero offset an inner product and its
        // masked sum on the key basis, one ModDown, the zero offset's product; its rescales
        const int lv = lp.level_in;
        const double nz = (double)lp.comb_shifts.size() - 1.0;
        bytes += modup(lv) + nz * (inner(lv) + limb * (3.0 * (lv + 1 + a) + 2.0 * (lv + 1))) + moddown(lv) +
                 limb * 4.0 * (lv + 1 + a) + mask(lv);
        for (int r = 0; r < lp.n_rescale_comb; ++r) bytes += rs(lv - r);
      } else {
        bytes += limb * l1 * 2.0 * (lp.f_in + lp.f_out);
        for (int r = 0; r < lp.n_rescale_comb; ++r) bytes += lp.f_out * rs(lp.level_in - r);
        for (int g = 0; g < np; ++g) {
          const int cols = std::min(lp.f_out, (g + 1) * lp.t) - g * lp.t;
          bytes += (cols - 1) * ks_single(la);
        }
      }
      if (lp.family == 3) {
        // radix-2 program: every term one masked product at its step's level, every
        // distinct (register, amount) one hoisted switch (one ModUp per register),
        // a rescale per register and per result level, the result terms summed
        const R2Program& r2 = lp.r2;
        double per = mask(la);
        std::set<std::pair<int, int64_t>> seen;
        std::set<int> upped;
        for (const R2Step& st : r2.steps) {
          const int lv = la - st.depth;
          for (const auto* v : {&st.keep, &st.fin})
            for (const R2Term& t : *v) {
              per += mask(lv);
              if (t.m && seen.insert({st.src, t.m}).second) {
                per += ks_extra(lv);
                if (upped.insert(st.src).second) per += modup(lv);
              }
            }
        }
        for (size_t r = 1; r < r2.reg_depth.size(); ++r) per += rs(la - r2.reg_depth[r] + 1);
        for (int d = 0; d < r2.depth; ++d) per += rs(la - d) + limb * 2.0 * (la - r2.depth + 1);
        bytes += np * per;
        n_out_cts = np;
        if (lp.act) bytes += n_out_cts * (ks_single(lp.level_out) + limb * 5.0 * (lp.level_out + 1));
        continue;
      }
      const size_t ns = lp.shifts.size();
      std::set<int64_t> babies, giants;
      for (int64_t d : lp.shifts) {
        int64_t q = d >= 0 ? d / lp.G : -((-d + lp.G - 1) / lp.G);
        if (d - q * lp.G) babies.insert(d - q * lp.G);
        if (q) giants.insert(q);
      }
      const double nz = (double)(ns - (std::count(lp.shifts.begin(), lp.shifts.end(), 0) ? 1 : 0));
      double per = mask(la) * ns + limb * 2.0 * (la + 1);
      if (lp.family == 1)
        per += modup(la) + nz * ks_extra(la);
      else if (lp.family == 4)   // inner products, their masked sum on the key basis, one ModDown
        per += modup(la) + nz * (inner(la) + limb * (3.0 * (la + 1 + a) + 2.0 * (la + 1))) + moddown(la) +
               limb * 4.0 * (la + 1 + a);
      else   // hoisted baby steps; giant steps summed on the key basis before one ModDown
        per += (babies.empty() ? 0.0 : modup(la) + babies.size() * ks_extra(la)) +
               giants.size() * (modup(la) + inner(la) + limb * (3.0 * (la + 1 + a) + 2.0 * (la + 1))) +
               (giants.empty() ? 0.0 : moddown(la) + limb * 4.0 * (la + 1 + a));
      bytes += np * (per + rs(la));
      n_out_cts = np;
    }
    if (lp.act) bytes += n_out_cts * (ks_single(lp.level_out) + limb * 5.0 * (lp.level_out + 1));
  }
  return bytes;
}

}  // namespace ficgcn

using namespace ficgcn;

static ficgcn_status search_status(const Error& e) {
  set_error(e.msg);
  return (ficgcn_status)e.code;
}

#define S_TRY try {
#define S_END                                           \
  return FICGCN_OK;                                     \
  }                                                     \
  catch (const Error& e) { return search_status(e); }   \
  catch (const std::exception& e) {                     \
    set_error(e.what());                                \
    return FICGCN_EINVAL;                               \
  }

extern "C" {

ficgcn_status ficgcn_plan_candidates(uint32_t n_v, const uint32_t* dims, uint32_t n_layers, uint32_t log_n,
                                     const ficgcn_plan_opts* base, ficgcn_plan_opts* out, size_t cap,
                                     size_t* n_out) {
  S_TRY
  if (!dims || !base || !n_out || n_v == 0 || n_layers == 0 || log_n < 2 || log_n > 20)
    FICGCN_THROW(EINVAL_, "bad argument");
  auto c = candidates(n_v, dims, n_layers, log_n, *base);
  *n_out = c.size();
  for (size_t i = 0; i < c.size() && i < cap && out; ++i) out[i] = c[i];
  S_END
}

ficgcn_status ficgcn_candidate_features(const int32_t* rowptr, const int32_t* col, uint32_t n_v, const uint32_t* dims,
                                        uint32_t n_layers, uint32_t log_n, const ficgcn_plan_opts* opts, float* out) {
  S_TRY
  if (!rowptr || !col || !dims || !opts || !out || n_v == 0 || n_layers == 0 || log_n < 2 || log_n > 20)
    FICGCN_THROW(EINVAL_, "bad argument");
  for (uint32_t v = 0; v < n_v; ++v)
    if (rowptr[v + 1] < rowptr[v]) FICGCN_THROW(EINVAL_, "rowptr not monotone");
  features(rowptr, col, n_v, dims, n_layers, log_n, *opts, out);
  S_END
}

ficgcn_status ficgcn_plan_cost(const ficgcn_plan* plan, double* bytes_out) {
  S_TRY
  if (!plan || !bytes_out) FICGCN_THROW(EINVAL_, "null argument");
  *bytes_out = plan_bytes(plan);
  S_END
}

ficgcn_status ficgcn_plan_search(ckks_ctx* ctx, const int32_t* rowptr, const int32_t* col, const double* val,
                                 uint32_t n_v, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                                 const ficgcn_plan_opts* base, ficgcn_mlp* model, uint32_t keep,
                                 ficgcn_plan_opts* best_out, ficgcn_search_stats* stats_out) {
  S_TRY
  if (!ctx || !rowptr || !col || !val || !dims || !weights || !base || !best_out || n_v == 0 || n_layers == 0)
    FICGCN_THROW(EINVAL_, "null or empty argument");
  auto cand = candidates(n_v, dims, n_layers, (uint32_t)ctx->log_n, *base);
  std::vector<size_t> order(cand.size());
  std::iota(order.begin(), order.end(), 0);
  size_t n_try = cand.size();
  if (model && keep > 0 && keep < cand.size()) {
    // predicted latency of every candidate, fastest first
    std::vector<float> feat(cand.size() * FICGCN_N_FEATURES);
    for (size_t i = 0; i < cand.size(); ++i)
      features(rowptr, col, n_v, dims, n_layers, (uint32_t)ctx->log_n, cand[i], feat.data() + i * FICGCN_N_FEATURES);
    ensure_device(ctx);
    float* xd = (float*)ctx->buf(65, feat.size() * 4);
    float* yd = (float*)ctx->buf(66, cand.size() * 4);
    HIPCHECK(hipMemcpyAsync(xd, feat.data(), feat.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    mlp_predict(model, xd, cand.size(), yd);
    std::vector<float> pred(cand.size());
    HIPCHECK(hipMemcpyAsync(pred.data(), yd, pred.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHECK(hipStreamSynchronize(ctx->stream));
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return pred[a] < pred[b]; });
    n_try = keep;
  }
  double best = 0;
  int best_i = -1;
  uint32_t built = 0, judged = 0;
  double secs = 0;
  // a key set of N words per limb, beta digits of 2 (L + alpha) limbs, per rotation step
  const double key_bytes = (double)((ctx->L + ctx->alpha - 1) / ctx->alpha) * 2.0 * (ctx->L + ctx->alpha) * ctx->N * 8.0;
  // candidates in order from lo, until `want` feasible ones are judged; a candidate that cannot be
  // built, or whose rotation keys exceed base->max_key_bytes, is infeasible
  auto judge = [&](size_t lo, size_t want) {
    for (size_t k = lo; k < cand.size() && judged < want; ++k) {
      const ficgcn_plan_opts& o = cand[order[k]];
      ficgcn_plan* p = nullptr;
      auto t0 = std::chrono::steady_clock::now();
      ficgcn_status st = ficgcn_plan_create(ctx, rowptr, col, val, n_v, dims, n_layers, weights, &o, &p);
      secs += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (st != FICGCN_OK) continue;   // infeasible candidate (e.g. the graph does not fit a block)
      ++built;
      size_t n_steps = 0;
      (void)ficgcn_plan_rot_steps(p, nullptr, 0, &n_steps);
      if (base->max_key_bytes > 0 && (double)n_steps * key_bytes > base->max_key_bytes) {
        ficgcn_plan_destroy(p);
        continue;
      }
      ++judged;
      const double b = plan_bytes(p);
      ficgcn_plan_destroy(p);
      if (best_i < 0 || b < best) {
        best = b;
        best_i = (int)order[k];
      }
    }
  };
  judge(0, n_try);
  if (best_i < 0) FICGCN_THROW(EPLAN_, "no candidate plan could be built");
  *best_out = cand[best_i];
  if (stats_out) {
    stats_out->n_candidates = (uint32_t)cand.size();
    stats_out->n_built = built;
    stats_out->best_cost = best;
    stats_out->build_seconds = secs;
  }
  S_END
}

}  // extern "C"
