// Planner of the encrypted GCN (host C++).
//
// Packing (paper Sec. 3.2, App. B): t feature columns per ciphertext, column
// c of a ciphertext in slots [c*B, (c+1)*B), B = M/t, node v at c*B + pi(v).
// Aggregation mode (Sec. 3.3.2): the first layer is Inter-CA over the
// client's neighbour copies; later layers are SpIntra-CA: combination first
// (one column per ciphertext), packing of t = min(pow2(F'), M / pow2(n_v))
// columns (t = 1 for every SpIntra-CA layer when one of them feeds another
// layer), then routing of every nonzero A_vu by its shift pi(u) - pi(v) in
// the diagonal form (one rotation + mask per distinct shift, all rotations
// hoisted on one ModUp), the baby-step/giant-step form, or the paper's
// radix-2 form with per-round masks (radix2.cpp).
// Node order (Sec. 3.4, Alg. 1): sibling-BFS regions of at most TH nodes
// (highest degree first; when the BFS runs dry the region continues from the
// highest-degree node left), interleaved round-robin (an exhausted region's
// turn takes a blank while blanks last), then greedy placement in BFS order
// where each node takes the free slot of its region adding the fewest shifts
// not yet used (lowest slot on ties).  With t = 1 shifts are taken mod M in
// (-M/2, M/2] (AOO, Sec. 3.3.1).
// Scale schedule: the scale is a double tracked through a fixed sequence of
// IEEE operations (first layer: sP = q_l, sW = q_{l-1}, two rescales; later
// layers: sW = (q_l [* q_{l-1}] * Delta) / s with one [two] rescale(s),
// masks at sM = q_l, one rescale; x^2 leaves its rescale to the consumer).
#include <algorithm>
#include <cmath>
#include <deque>
#include <set>

#include "../../include/ficgcn.h"
#include "plan.h"

namespace ficgcn {

static int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}
static int64_t fmod_(int64_t a, int64_t b) { return a - fdiv(a, b) * b; }

static int next_pow2(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}

static int64_t reduce_shift(int64_t d, int64_t M, bool wrap) {
  if (!wrap) return d;
  int64_t r = fmod_(d, M);
  return r > M / 2 ? r - M : r;
}

static int clog2(int64_t x) {
  int r = 0;
  while (((int64_t)1 << r) < x) ++r;
  return r;
}

// J(t; F, n) = 2 ceil(F n / t) + 20 ceil(log2 t)  (Sec. 3.2 case M > N F', App. B)
static int64_t j_objective(int64_t t, int64_t F, int64_t n) { return 2 * ((F * n + t - 1) / t) + 20 * clog2(t); }

// The paper's t: the argmin of J over powers of two with t N F' <= M (ties -> smaller t);
// 1 when M <= N F' (case 2)
static int paper_packing_t(int64_t F, int64_t n, int64_t N, int64_t Fo, int64_t M) {
  if (M <= N * Fo) return 1;
  int64_t best = 1, bj = j_objective(1, F, n);
  for (int64_t t = 2; t * N * Fo <= M; t *= 2) {
    int64_t j = j_objective(t, F, n);
    if (j < bj) {
      best = t;
      bj = j;
    }
  }
  return (int)best;
}

// node block of the case-1 layout: M / (t pow2(F')), or 0 when pow2(N) does not fit it
static int rep_block(int t, int Fo, int N, int M) {
  if (t < 1 || Fo < 1) return 0;
  const int Bc = M / (t * next_pow2(Fo));
  return Bc >= next_pow2(N) ? Bc : 0;
}

// the first layer's packing by the paper's rule on the case-1 layout: t > 0 (that layout) or
// 0 (one column per ciphertext); t halved while the layout or a later width does not fit
static int rule_packing(int F, int n, int N, int Fo, int M, const std::vector<int>& later) {
  if ((int64_t)M <= (int64_t)N * Fo) return 0;
  for (int t = paper_packing_t(F, n, N, Fo, M); t >= 1; t /= 2) {
    const int Bc = rep_block(t, Fo, N, M);
    bool ok = Bc > 0;
    for (int f : later) ok = ok && f <= M / std::max(Bc, 1);
    if (ok) return t;
  }
  return 0;
}

// Sec. 3.3.2: Inter-CA 2 ceil(F n / t) against SpIntra-CA 10 c n log2(N)^2
static void mode_costs(LayerPlan& lp, int n, int t, int N, double c) {
  lp.mode_cost_inter = (double)(2 * (((int64_t)lp.f_in * n + t - 1) / t));
  const double lg = std::log2((double)std::max(N, 2));
  lp.mode_cost_spintra = 10.0 * c * n * (lg * lg);
  lp.paper_mode = lp.mode_cost_inter <= lp.mode_cost_spintra ? 0 : 1;
}

struct Rows {
  int n;
  const std::vector<int32_t>& rp;
  const std::vector<int32_t>& col;
};

static std::vector<std::vector<int>> regions_of(const ficgcn_plan* p, int TH) {
  const int n = p->n_v;
  std::vector<std::set<int>> sup(n), sib(n);
  for (int v = 0; v < n; ++v) {
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e) {
      int u = p->col[e];
      if (u != v) {
        sup[v].insert(u);
        sup[u].insert(v);
      }
      for (int e2 = p->rowptr[v]; e2 < p->rowptr[v + 1]; ++e2) sib[u].insert(p->col[e2]);
    }
  }
  std::vector<std::vector<int>> sibv(n);
  for (int x = 0; x < n; ++x) {
    sib[x].erase(x);
    sibv[x].assign(sib[x].begin(), sib[x].end());
  }
  std::vector<int> order(n);
  for (int v = 0; v < n; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (sup[a].size() != sup[b].size()) return sup[a].size() > sup[b].size();
    return a < b;
  });
  std::vector<char> remaining(n, 1);
  std::vector<std::vector<int>> regions;
  size_t ptr = 0;
  int n_left = n;
  while (n_left > 0) {
    std::vector<int> region;
    std::set<int> visited;
    while ((int)region.size() < TH && n_left > 0) {
      while (!remaining[order[ptr]]) ++ptr;
      int start = order[ptr];
      std::deque<int> q{start};
      visited.insert(start);
      while (!q.empty() && (int)region.size() < TH) {
        int x = q.front();
        q.pop_front();
        region.push_back(x);
        remaining[x] = 0;
        --n_left;
        for (int w : sibv[x])
          if (remaining[w] && !visited.count(w)) {
            visited.insert(w);
            q.push_back(w);
          }
      }
    }
    regions.push_back(region);
  }
  return regions;
}

static std::vector<std::vector<int>> interleave(const std::vector<int>& sizes, int B) {
  const int R = (int)sizes.size();
  std::vector<int> left(sizes);
  int total = 0;
  for (int s : sizes) total += s;
  int blanks = B - total;
  if (blanks < 0) FICGCN_THROW(EPLAN_, "graph does not fit the column block");
  std::vector<std::vector<int>> slots(R);
  int j = 0;
  auto any = [&] {
    for (int x : left)
      if (x > 0) return true;
    return false;
  };
  while (any()) {
    for (int r = 0; r < R; ++r) {
      if (left[r] > 0) {
        slots[r].push_back(j++);
        --left[r];
      } else if (blanks > 0) {
        --blanks;
        ++j;
      }
    }
  }
  return slots;
}

// Stage 3: greedy placement in BFS order, each node at the free slot of its region with
// the least cost (ties -> lowest slot).  conflicts = false: the shifts the node's demands
// add to the plan (the diagonal and baby-step/giant-step forms pay per distinct shift);
// conflicts = true (the radix-2 form): the (round, slot) cells where the node's demands
// with placed nodes meet a placed demand of another source.  A radix-2 demand from slot s
// with shift d sits, after each round r below the highest bit of |d|, at
// s - sign(d) (|d| mod 2^(r+1)) (mod M); in its last round it arrives and leaves.
static void place(ficgcn_plan* p, const std::vector<std::vector<int>>& regions,
                  const std::vector<std::vector<int>>& slots, bool wrap, bool conflicts) {
  const int n = p->n_v;
  const int64_t M = p->M;
  std::vector<std::vector<int>> out_nb(n), in_nb(n);
  for (int v = 0; v < n; ++v)
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e) {
      int u = p->col[e];
      if (u != v) {
        out_nb[v].push_back(u);
        in_nb[u].push_back(v);
      }
    }
  p->pi.assign(n, -1);
  // shifts lie in (-M, M): index d + M
  std::vector<char> used(2 * M + 1, 0);
  std::vector<int> stamp(2 * M + 1, -1);
  int R = 0;
  while ((M >> R) > 0) ++R;   // bit length of M
  // source node per (round, slot); -1 free, -2 several sources
  std::vector<int> occ(conflicts ? (size_t)R * M : 0, -1);
  auto red = [&](int64_t d) { return reduce_shift(d, M, wrap); };
  auto cell = [&](int64_t s, int64_t d, int r) {
    const int64_t mag = d < 0 ? -d : d, part = mag % ((int64_t)1 << (r + 1));
    int64_t c = (s - (d > 0 ? part : -part)) % M;
    return (size_t)r * M + (size_t)(c < 0 ? c + M : c);
  };
  auto travels = [](int64_t d, int r) { return ((d < 0 ? -d : d) >> (r + 1)) != 0; };
  auto occupy = [&](int src, int64_t s, int64_t d) {
    for (int r = 0; r < R && travels(d, r); ++r) {
      int& o = occ[cell(s, d, r)];
      o = o == -1 ? src : (o == src ? o : -2);
    }
  };
  auto add_shifts = [&](int x) {
    for (int u : out_nb[x])
      if (p->pi[u] >= 0) {
        const int64_t d = red((int64_t)p->pi[u] - p->pi[x]);
        used[d + M] = 1;
        if (conflicts) occupy(u, p->pi[u], d);
      }
    for (int v : in_nb[x])
      if (p->pi[v] >= 0) {
        const int64_t d = red((int64_t)p->pi[x] - p->pi[v]);
        used[d + M] = 1;
        if (conflicts) occupy(x, p->pi[x], d);
      }
  };
  auto walk_cost = [&](int src, int64_t s, int64_t d) {
    long c = 0;
    for (int r = 0; r < R && travels(d, r); ++r) {
      const int o = occ[cell(s, d, r)];
      c += (o != -1 && o != src) ? 1 : 0;
    }
    return c;
  };
  int stamp_id = 0;
  for (size_t r = 0; r < regions.size(); ++r) {
    const std::vector<int>& reg = regions[r];
    const std::vector<int>& sl = slots[r];
    std::vector<char> taken(sl.size(), 0);
    p->pi[reg[0]] = sl[0];
    taken[0] = 1;
    add_shifts(reg[0]);
    for (size_t idx = 1; idx < reg.size(); ++idx) {
      int x = reg[idx];
      std::vector<int> pu, pv, su;
      for (int u : out_nb[x])
        if (p->pi[u] >= 0) {
          pu.push_back(p->pi[u]);
          su.push_back(u);
        }
      for (int v : in_nb[x])
        if (p->pi[v] >= 0) pv.push_back(p->pi[v]);
      int best = -1;
      long best_cost = -1;
      for (size_t k = 0; k < sl.size(); ++k) {
        if (taken[k]) continue;
        int64_t pos = sl[k];
        long cost = 0;
        if (conflicts) {
          for (size_t a = 0; a < pu.size(); ++a) cost += walk_cost(su[a], pu[a], red(pu[a] - pos));
          for (int b : pv) cost += walk_cost(x, pos, red(pos - b));
        } else if (!pu.empty() || !pv.empty()) {
          ++stamp_id;
          for (int a : pu) {
            int64_t d = red(a - pos) + M;
            if (!used[d] && stamp[d] != stamp_id) {
              stamp[d] = stamp_id;
              ++cost;
            }
          }
          for (int b : pv) {
            int64_t d = red(pos - b) + M;
            if (!used[d] && stamp[d] != stamp_id) {
              stamp[d] = stamp_id;
              ++cost;
            }
          }
        }
        if (best < 0 || cost < best_cost) {
          best = (int)k;
          best_cost = cost;
          if (cost == 0) break;   // lowest free slot with zero cost
        }
      }
      p->pi[x] = sl[best];
      taken[best] = 1;
      add_shifts(x);
    }
  }
}

static void bsgs_split(const std::vector<int64_t>& shifts, int B, int& G_out, int& c_out) {
  int bestc = -1, bestG = 1;
  for (int64_t G = 1; G <= std::max(B, 1); G *= 2) {
    std::set<int64_t> babies, giants;
    for (int64_t d : shifts) {
      int64_t b = fmod_(d, G), g = fdiv(d, G);
      if (b) babies.insert(b);
      if (g) giants.insert(g);
    }
    int c = (int)(babies.size() + giants.size());
    if (bestc < 0 || c < bestc) {
      bestc = c;
      bestG = (int)G;
    }
  }
  G_out = bestG;
  c_out = bestc;
}

static std::vector<int64_t> rotation_steps_of(const LayerPlan& lp) {
  std::set<int64_t> s;
  if (lp.family == 3) {
    for (const R2Step& st : lp.r2.steps) {
      for (const R2Term& t : st.keep)
        if (t.m) s.insert(t.m);
      for (const R2Term& t : st.fin)
        if (t.m) s.insert(t.m);
    }
  } else if (lp.family == 1 || lp.family == 4) {
    for (int64_t d : lp.shifts)
      if (d) s.insert(d);
  } else {
    for (int64_t d : lp.shifts) {
      int64_t b = fmod_(d, lp.G), g = fdiv(d, lp.G) * lp.G;
      if (b) s.insert(b);
      if (g) s.insert(g);
    }
  }
  return std::vector<int64_t>(s.begin(), s.end());
}

// levels the layers consume: Inter-CA 2 (integer-weight combination) or 1 (case-1 layout),
// SpIntra-CA 1 or 2 combination rescales (2 after a squared input) plus 1 mask level (the
// radix-2 program: its depth)
static int levels_needed(const ficgcn_plan* p) {
  int need = 0;
  bool pending = false;
  for (const LayerPlan& lp : p->layers) {
    if (lp.kind == 0)
      need += lp.pack ? 1 : 2;
    else
      need += (pending ? 2 : 1) + (lp.family == 3 ? lp.r2.depth : 1);
    pending = lp.act;
  }
  return need;
}

static constexpr int OUT_LEVEL = 1;   // the output keeps two primes (scale Delta^2 after x^2)

static void schedule(ckks_ctx* c, ficgcn_plan* p) {
  const double delta = std::ldexp(1.0, c->log_scale);
  double s = delta;
  int lv = c->L - 1;
  if (p->low_level) lv = std::min(lv, levels_needed(p) + OUT_LEVEL);
  bool pending = false;
  for (LayerPlan& lp : p->layers) {
    lp.level_in = lv;
    lp.scale_in = s;
    if (lp.kind == 0 && lp.pack) {
      // case-1 layout: the operands carry A_hat_k (x) W, one level
      if (lv < 1) FICGCN_THROW(EPLAN_, "not enough levels for the Inter-CA layer");
      lp.sP = (double)c->mod[lv];
      lp.sW = 0.0;
      s = s * lp.sP;
      s = s / (double)c->mod[lv];
      lv -= 1;
      lp.op_level = lp.level_in;
      lp.op_scale = lp.sP;
    } else if (lp.kind == 0) {
      if (lv < 2) FICGCN_THROW(EPLAN_, "not enough levels for the Inter-CA layer");
      lp.sP = (double)c->mod[lv];
      lp.sW = (double)c->mod[lv - 1];
      s = s * lp.sP;
      s = s * lp.sW;
      s = s / (double)c->mod[lv];
      s = s / (double)c->mod[lv - 1];
      lv -= 2;
      lp.op_level = lp.level_in;
      lp.op_scale = lp.sP;
    } else {
      lp.n_rescale_comb = pending ? 2 : 1;
      if (lv < lp.n_rescale_comb + 1) FICGCN_THROW(EPLAN_, "not enough levels for the SpIntra-CA layer");
      if (pending) {
        lp.sW = (((double)c->mod[lv] * (double)c->mod[lv - 1]) * delta) / s;
        s = s * lp.sW;
        s = s / (double)c->mod[lv];
        s = s / (double)c->mod[lv - 1];
        lv -= 2;
      } else {
        lp.sW = ((double)c->mod[lv] * delta) / s;
        s = s * lp.sW;
        s = s / (double)c->mod[lv];
        lv -= 1;
      }
      lp.level_agg = lv;
      lp.scale_agg = s;
      lp.sM = (double)c->mod[lv];
      if (lp.family == 3) {
        // every step's masks are encoded at the prime its rescale drops: the
        // result keeps the scale exactly; one level per step on the deepest chain
        if (lv < lp.r2.depth) FICGCN_THROW(EPLAN_, "not enough levels for the radix-2 aggregation");
        lv -= lp.r2.depth;
      } else {
        s = s * lp.sM;
        s = s / (double)c->mod[lv];
        lv -= 1;
      }
      lp.op_level = lp.level_agg;
      lp.op_scale = lp.sM;
    }
    pending = false;
    if (lp.act) {
      s = s * s;
      pending = true;
    }
    lp.squared_out = pending;
    lp.level_out = lv;
    lp.scale_out = s;
  }
}

size_t LayerPlan::n_agg_ops() const {
  if (kind == 0) return 0;
  if (family == 3) return (size_t)n_packed() * r2.ops.size();
  return (size_t)n_packed() * shifts.size();
}

// Operands of a layer, in order: Inter-CA: the K copies' adjacency plaintexts, or, in the
// case-1 layout, K * ceil(F / t) plaintexts (copy k, input ciphertext j at k * J + j);
// SpIntra-CA: the aggregation masks (packed ciphertext g, then shift or program operand),
// then, for the block-rotation combination, one mask per block offset (comb_shifts order)
size_t plan_operand_count(const ficgcn_plan* p, int li) {
  const LayerPlan& lp = p->layers[li];
  if (lp.kind == 0) return lp.pack ? (size_t)lp.n_in_cts() : (size_t)lp.K;
  return lp.n_agg_ops() + (lp.comb ? lp.comb_shifts.size() : 0);
}

static bool is_comb_operand(const LayerPlan& lp, size_t i) { return lp.kind == 1 && lp.comb && i >= lp.n_agg_ops(); }

int plan_operand_level(const ficgcn_plan* p, int li, size_t i) {
  const LayerPlan& lp = p->layers[li];
  if (is_comb_operand(lp, i)) return lp.level_in;
  if (lp.kind == 1 && lp.family == 3) return lp.level_agg - lp.r2.ops[i % lp.r2.ops.size()].depth;
  return lp.op_level;
}

double plan_operand_scale(const ficgcn_plan* p, int li, size_t i) {
  const LayerPlan& lp = p->layers[li];
  if (is_comb_operand(lp, i)) return lp.sW;
  if (lp.kind == 1 && lp.family == 3) return (double)p->ctx->mod[plan_operand_level(p, li, i)];
  return lp.op_scale;
}

bool plan_operand_ext(const ficgcn_plan* p, int li, size_t i) {
  const LayerPlan& lp = p->layers[li];
  if (is_comb_operand(lp, i)) return lp.comb_shifts[i - lp.n_agg_ops()] != 0;
  return lp.kind == 1 && lp.family == 4;
}

static void layout_operands(ficgcn_plan* p) {
  const size_t N = p->ctx->N;
  for (size_t li = 0; li < p->layers.size(); ++li) {
    LayerPlan& lp = p->layers[li];
    const size_t n = plan_operand_count(p, (int)li);
    lp.op_x.resize(n);
    lp.op_lv.resize(n);
    lp.op_off.resize(n);
    lp.op_alias.assign(n, -1);
    // aggregation masks depend on the packed ciphertext only through its column count
    // (mask slots c B + pi(v) for c < n_cols): packed ciphertexts with the first one's
    // count share its masks
    const size_t nag = lp.n_agg_ops(), np = lp.kind == 1 ? (size_t)lp.n_packed() : 1;
    const size_t per = np ? nag / np : 0;
    const int cols0 = std::min(lp.t, lp.f_out);
    size_t off = 0;
    for (size_t i = 0; i < n; ++i) {
      lp.op_x[i] = plan_operand_ext(p, (int)li, i) ? 1 : 0;
      lp.op_lv[i] = plan_operand_level(p, (int)li, i);
      if (i < nag && per && i >= per) {
        const int g = (int)(i / per);
        if (std::min(lp.t, lp.f_out - g * lp.t) == cols0) {
          lp.op_alias[i] = (int32_t)(i % per);
          lp.op_off[i] = lp.op_off[i % per];
          continue;
        }
      }
      lp.op_off[i] = off;
      off += (size_t)(lp.op_lv[i] + 1 + (lp.op_x[i] ? p->ctx->alpha : 0)) * N;
    }
    lp.op_words = off;
  }
}

// first slot of the block of input column b and output column l in the case-1 layout
static size_t rep_slot(const LayerPlan& lp, int b, int l) { return ((size_t)b * next_pow2(lp.f_out) + l) * lp.B; }

void plan_operand_slots(const ficgcn_plan* p, int li, size_t i, std::vector<double>& out) {
  const LayerPlan& lp = p->layers[li];
  const int M = p->M, n = p->n_v;
  out.assign(M, 0.0);
  if (lp.kind == 0 && lp.pack) {
    // A_hat[v, src_k(v)] * W[j t + b, l] at rep_slot(b, l) + pi(v)
    const int J = (lp.f_in + lp.t - 1) / lp.t;
    const int k = (int)(i / J), j = (int)(i % J);
    for (int b = 0; b < lp.t && j * lp.t + b < lp.f_in; ++b) {
      const int f = j * lp.t + b;
      for (int l = 0; l < lp.f_out; ++l) {
        const double wv = lp.w[(size_t)f * lp.f_out + l];
        const size_t base = rep_slot(lp, b, l);
        for (int v = 0; v < n; ++v)
          if (lp.copy_src[(size_t)k * n + v] >= 0) out[base + p->pi[v]] = lp.copy_val[(size_t)k * n + v] * wv;
      }
    }
    return;
  }
  if (lp.kind == 0) {
    for (int v = 0; v < n; ++v)
      if (lp.copy_src[i * n + v] >= 0) out[p->pi[v]] = lp.copy_val[i * n + v];
    return;
  }
  if (is_comb_operand(lp, i)) {
    // block offset s: cm_s[c B + pi(v)] = W[c + s, c]
    const int64_t s = lp.comb_shifts[i - lp.n_agg_ops()];
    for (int c = 0; c < lp.f_out; ++c) {
      const int64_t l = c + s;
      if (l < 0 || l >= lp.f_in) continue;
      const double wv = lp.w[(size_t)l * lp.f_out + c];
      for (int v = 0; v < n; ++v) out[(size_t)c * lp.B + p->pi[v]] = wv;
    }
    return;
  }
  if (lp.family == 3) {
    const size_t nops = lp.r2.ops.size();
    const int g = (int)(i / nops);
    const int n_cols = std::min(lp.t, lp.f_out - g * lp.t);
    const R2Program::Ref& ref = lp.r2.ops[i % nops];
    const R2Term* t = &lp.r2.self;
    if (ref.step >= 0) {
      const R2Step& st = lp.r2.steps[ref.step];
      t = ref.term < (int)st.keep.size() ? &st.keep[ref.term] : &st.fin[ref.term - st.keep.size()];
    }
    for (size_t k = 0; k < t->slot.size(); ++k)
      for (int cc = 0; cc < n_cols; ++cc) out[(size_t)cc * lp.B + t->slot[k]] = t->val[k];
    return;
  }
  const size_t ns = lp.shifts.size();
  const int g = (int)(i / ns);
  const int64_t delta = lp.shifts[i % ns];
  const int n_cols = std::min(lp.t, lp.f_out - g * lp.t);
  const bool wrap = lp.B == M;
  std::vector<double> mask(M, 0.0);
  for (int v = 0; v < n; ++v)
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e) {
      int u = p->col[e];
      if (reduce_shift((int64_t)p->pi[u] - p->pi[v], M, wrap) != delta) continue;
      for (int cc = 0; cc < n_cols; ++cc) mask[(size_t)cc * lp.B + p->pi[v]] = p->val[e];
    }
  if (lp.family == 2) {
    // pre-rotated by -g*G: out[i] = mask[(i - gG) mod M]
    int64_t gG = fdiv(delta, lp.G) * lp.G;
    for (int64_t k = 0; k < M; ++k) out[k] = mask[fmod_(k - gG, M)];
  } else {
    out = mask;
  }
}

}  // namespace ficgcn

using namespace ficgcn;

ficgcn_plan::~ficgcn_plan() {
  if (ctx && ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ficgcn::release_plan_device(this);
}

namespace ficgcn {

LayerGraph::~LayerGraph() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
}

void release_plan_device(ficgcn_plan* p) {
  p->graphs.clear();
  for (auto& lp : p->layers) {
    for (void** q : {(void**)&lp.ops_block, (void**)&lp.w_dev, &lp.wf_dev, (void**)&lp.wm_dev, (void**)&lp.pw_dev})
      if (*q) {
        (void)hipFree(*q);
        *q = nullptr;
      }
    for (auto& o : lp.ops) o = nullptr;
    lp.wm_state = 0;
  }
}

size_t plan_operand_bytes(const ficgcn_plan* p) {
  size_t b = 0;
  for (const auto& lp : p->layers) b += lp.op_words * 8;
  return b;
}

}  // namespace ficgcn

namespace ficgcn {

static void inter_copies(const ficgcn_plan* p, LayerPlan& lp, int K) {
  const int n = p->n_v;
  lp.K = K;
  lp.copy_src.assign((size_t)lp.K * n, -1);
  lp.copy_val.assign((size_t)lp.K * n, 0.0);
  for (int v = 0; v < n; ++v) {
    int k = 1;
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e) {
      int u = p->col[e];
      if (u == v) {
        lp.copy_src[v] = v;
        lp.copy_val[v] = p->val[e];
      } else {
        lp.copy_src[(size_t)k * n + v] = u;
        lp.copy_val[(size_t)k * n + v] = p->val[e];
        ++k;
      }
    }
  }
}

// routing of a SpIntra-CA layer on blocks of B slots
static void spintra_routing(const ficgcn_plan* p, LayerPlan& lp, int B, const ficgcn_plan_opts& o) {
  const int n = p->n_v, M = p->M;
  lp.B = B;
  lp.t = M / B;
  const bool wrap = lp.B == M;
  std::set<int64_t> sh;
  for (int v = 0; v < n; ++v)
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e)
      sh.insert(reduce_shift((int64_t)p->pi[p->col[e]] - p->pi[v], M, wrap));
  lp.shifts.assign(sh.begin(), sh.end());
  int c2;
  bsgs_split(lp.shifts, lp.B, lp.G, c2);
  int c1 = (int)lp.shifts.size() - (sh.count(0) ? 1 : 0);
  lp.family = (o.family >= 1 && o.family <= 4) ? o.family : (c2 < c1 ? 2 : 1);
  if (lp.family == 3) {
    if (!(o.cpoo >= 0.0 && o.cpoo <= 1.0)) FICGCN_THROW(EPLAN_, "CPOO threshold must lie in [0, 1]");
    lp.cpoo = o.cpoo;
    build_radix2(p->pi, p->rowptr, p->col, p->val, M, lp.B, wrap && !o.aoo_off, o.cpoo, lp.r2);
  }
}

static void schedule(ckks_ctx* c, ficgcn_plan* p);
static void layout_operands(ficgcn_plan* p);
static std::vector<int64_t> rotation_steps_of(const LayerPlan& lp);

// node order over blocks of B slots (Alg. 1, or the identity)
static void node_order(ficgcn_plan* p, int B, const ficgcn_plan_opts& o) {
  const int n = p->n_v;
  p->B_pi = B;
  const int TH = o.TH > 0 ? o.TH : (n < 10000 ? 1024 : 4096);
  if (o.use_noo) {
    p->regions = regions_of(p, TH);
    std::vector<int> sizes;
    for (auto& r : p->regions) sizes.push_back((int)r.size());
    auto slots = interleave(sizes, B);
    place(p, p->regions, slots, B == p->M, o.family == 3);
  } else {
    if (n > B) FICGCN_THROW(EPLAN_, "graph does not fit the column block");
    p->pi.resize(n);
    for (int v = 0; v < n; ++v) p->pi[v] = v;
    p->regions = {std::vector<int>()};
    for (int v = 0; v < n; ++v) p->regions[0].push_back(v);
  }
}

static void finish_plan(ckks_ctx* c, ficgcn_plan* p, const double* const* weights) {
  schedule(c, p);
  layout_operands(p);
  for (size_t li = 0; li < p->layers.size(); ++li) {
    LayerPlan& lp = p->layers[li];
    lp.w.assign(weights[li], weights[li] + (size_t)lp.f_in * lp.f_out);
    lp.w_int.resize((size_t)lp.f_in * lp.f_out);
    for (size_t i = 0; i < lp.w_int.size(); ++i) {
      double x = weights[li][i] * lp.sW;
      if (!(std::fabs(x) < 9.2e18)) FICGCN_THROW(ESCALE_, "weight times scale exceeds 63 bits");
      lp.w_int[i] = (int64_t)std::nearbyint(x);
    }
  }
  std::set<int64_t> steps;
  const int M = p->M;
  for (auto& lp : p->layers) {
    for (int64_t s : lp.fold_steps) steps.insert(fmod_(s, M));
    for (int64_t s : lp.comb_shifts) steps.insert(fmod_(s * lp.B, M));
    if (lp.kind != 1) continue;
    for (int64_t s : lp.pack_steps) steps.insert(fmod_(s, M));
    for (int64_t s : rotation_steps_of(lp)) steps.insert(fmod_(s, M));
  }
  steps.erase(0);
  p->rot_steps.assign(steps.begin(), steps.end());
}

// Inter-CA first layer in the case-1 layout at packing t1; every later layer SpIntra-CA on
// the packed blocks with the block-rotation combination
static void build_rep_plan(ckks_ctx* c, ficgcn_plan* p, const uint32_t* dims, uint32_t n_layers,
                           const double* const* weights, const ficgcn_plan_opts& o, int t1, int K) {
  const int M = p->M;
  const int Bc = rep_block(t1, (int)dims[1], p->n_v, M);
  if (!Bc) FICGCN_THROW(EPLAN_, "the case-1 layout does not fit at t = " + std::to_string(t1));
  node_order(p, Bc, o);
  const double agg_c = o.agg_c > 0 ? o.agg_c : 1.0;
  p->layers.clear();
  LayerPlan l0;
  l0.kind = 0;
  l0.f_in = (int)dims[0];
  l0.f_out = (int)dims[1];
  l0.act = o.activation != 0;
  inter_copies(p, l0, K);
  l0.pack = 1;
  l0.t = t1;
  l0.B = Bc;
  const int64_t S = (int64_t)next_pow2(l0.f_out) * Bc;
  for (int i = 0; (1 << i) < t1; ++i) l0.fold_steps.push_back(((int64_t)1 << i) * S);
  p->layers.push_back(l0);
  for (uint32_t li = 1; li < n_layers; ++li) {
    LayerPlan lp;
    lp.kind = 1;
    lp.f_in = (int)dims[li];
    lp.f_out = (int)dims[li + 1];
    lp.act = o.activation != 0;
    if (lp.f_out > M / Bc) FICGCN_THROW(EPLAN_, "a later layer is wider than the packed blocks hold");
    spintra_routing(p, lp, Bc, o);
    lp.comb = 1;
    for (int s = -(lp.f_out - 1); s < lp.f_in; ++s) lp.comb_shifts.push_back(s);
    mode_costs(lp, K - 1, lp.t, p->n_v, agg_c);
    p->layers.push_back(lp);
  }
  finish_plan(c, p, weights);
}

void build_plan(ckks_ctx* c, ficgcn_plan* p, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                const ficgcn_plan_opts& o) {
  const int n = p->n_v;
  const int M = c->N / 2;
  p->M = M;
  p->low_level = o.low_level != 0;
  if (o.first_mode == 1 && n_layers > 1)
    FICGCN_THROW(EPLAN_, "a SpIntra-CA first layer is only supported for one-layer models");
  int K_all = 0;
  for (int v = 0; v < n; ++v) {
    int off = 0;
    for (int e = p->rowptr[v]; e < p->rowptr[v + 1]; ++e) off += p->col[e] != v;
    K_all = std::max(K_all, off);
  }
  K_all += 1;
  if (o.first_mode == 0 && o.first_pack != 0) {
    std::vector<int> later(dims + 2, dims + n_layers + 1);
    int t1 = o.first_pack;
    if (t1 < 0) {
      t1 = rule_packing((int)dims[0], K_all - 1, n, (int)dims[1], M, later);
    } else {
      const int Bc = (t1 & (t1 - 1)) ? 0 : rep_block(t1, (int)dims[1], n, M);
      bool ok = Bc > 0;
      for (int f : later) ok = ok && f <= M / std::max(Bc, 1);
      if (!ok) FICGCN_THROW(EPLAN_, "the case-1 layout does not fit at t = " + std::to_string(t1));
    }
    if (t1 > 0) {
      build_rep_plan(c, p, dims, n_layers, weights, o, t1, K_all);
      return;
    }
  }
  std::vector<int> spin_f;
  bool chained = false;     // a SpIntra-CA layer feeds another layer: its outputs stay one column each
  for (uint32_t i = 0; i < n_layers; ++i)
    if (i > 0 || o.first_mode == 1) {
      spin_f.push_back((int)dims[i + 1]);
      chained |= i + 1 < n_layers;
    }
  int t_pack = 1;
  if (!spin_f.empty()) {
    t_pack = M / next_pow2(n);
    for (int f : spin_f) t_pack = std::min(t_pack, next_pow2(f));
  }
  if (chained) t_pack = 1;
  if (t_pack < 1) FICGCN_THROW(EPLAN_, "graph larger than the slot count");
  if (o.t != 0 && !spin_f.empty()) {
    if (o.t < 1 || (o.t & (o.t - 1)) || o.t > t_pack)
      FICGCN_THROW(EPLAN_, "packing t must be a power of two no larger than " + std::to_string(t_pack));
    t_pack = o.t;
  }
  const int B = M / t_pack;
  node_order(p, B, o);
  const double agg_c = o.agg_c > 0 ? o.agg_c : 1.0;
  p->layers.clear();
  for (uint32_t li = 0; li < n_layers; ++li) {
    LayerPlan lp;
    lp.f_in = (int)dims[li];
    lp.f_out = (int)dims[li + 1];
    lp.act = o.activation != 0;
    lp.kind = (li == 0 && o.first_mode == 0) ? 0 : 1;
    if (lp.kind == 0) {
      inter_copies(p, lp, K_all);
    } else {
      spintra_routing(p, lp, M / t_pack, o);
      if (li > 0) mode_costs(lp, K_all - 1, 1, n, agg_c);
      std::set<int64_t> pk;
      for (int l = 0; l < lp.f_out; ++l)
        if (l % lp.t) pk.insert(-(int64_t)(l % lp.t) * lp.B);
      lp.pack_steps.assign(pk.begin(), pk.end());
    }
    p->layers.push_back(lp);
  }
  finish_plan(c, p, weights);
}

std::vector<int64_t> layer_rotation_steps(const LayerPlan& lp) { return rotation_steps_of(lp); }

}  // namespace ficgcn
