// Radix-2 SpIntra-CA program (paper Sec. 3.3) with CPOO (Sec. 3.3.1), host side.
//
// A demand u -> v with coefficient A_vu carries the value at slot pi(u) to
// slot pi(v); its shift delta = pi(u) - pi(v) (AOO-reduced when t = 1) is
// travelled bit by bit: in round r every demand whose |delta| has bit r set
// moves by sign * 2^r.  A working ciphertext C takes one round as
//   C' = sum_m Rot(C, m) (.) Keep_m        (m in {0, +2^r, -2^r}; masks after
// the rotations, so the rotations of C share one ModUp), then a rescale.  A
// demand arriving in round r leaves C: Result += Rot(C, m) (.) Fin_m with its
// coefficient; self loops are the input times Fin_0.
//
// Working ciphertexts ("lanes"): demands in neighbour-index order (each
// row's non-self entries sorted by (|delta|, delta); the k-th of every row,
// rows ascending, before the (k+1)-th) go first-fit into the lanes where no
// slot, after any round in which they still travel, would hold values of two
// source nodes.  Every lane starts as the input ciphertext.  A lane skips a
// round in which none of its demands moves.
//
// CPOO with threshold theta: a lane is sparse when its live slots are fewer
// than theta * B.  At boundary r (a) the demands a sparse lane carries past
// round r move, slot by slot, into the first earlier non-sparse lane of the
// same level that steps in round r, where their slot after round r is free
// and no later slot conflicts; the sparse lane's step writes them into that
// lane's next ciphertext; (b) what a sparse lane keeps runs the rounds
// r .. r+w-1 as one step (demand amounts sign * (|delta| mod 2^(r+w) -
// |delta| mod 2^r)), w the longest window whose distinct nonzero amounts are
// no more than the rotations of its rounds taken one by one.
#include <algorithm>
#include <map>
#include <set>
#include <unordered_map>

#include "plan.h"

namespace ficgcn {
namespace {

struct Dm {
  int32_t u, v;
  int64_t s, e;       // source and target slot (block-local)
  int64_t delta, mag;
  int sign, hb;       // hb: highest set bit of |delta| = the round of arrival
  double a;
};

int64_t mod_pos(int64_t x, int64_t M) {
  x %= M;
  return x < 0 ? x + M : x;
}

// slot after round r (r = -1: the source)
int64_t slot_after(const Dm& d, int r, int64_t M) {
  if (r < 0) return d.s;
  return mod_pos(d.s - d.sign * (d.mag & ((int64_t(1) << (r + 1)) - 1)), M);
}

// signed amount travelled in rounds [r, r + w)
int64_t amount(const Dm& d, int r, int w) {
  const int64_t hi = d.mag & ((int64_t(1) << (r + w)) - 1);
  const int64_t lo = d.mag & ((int64_t(1) << r) - 1);
  return d.sign * (hi - lo);
}

uint64_t okey(int r, int64_t slot) { return ((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)slot; }

using Occ = std::unordered_map<uint64_t, int32_t>;

struct Lane {
  std::vector<int> dm;     // demand indices
  Occ occ;                 // (round, slot) -> source node while travelling
  int reg = 0, depth = 0, bnd = 0;
};

void occupy(Occ& o, const Dm& d, int64_t M) {
  for (int r = 0; r < d.hb; ++r) o[okey(r, slot_after(d, r, M))] = d.u;
}

bool fits(const Occ& o, const Dm& d, int from, int64_t M) {
  for (int r = from; r < d.hb; ++r) {
    auto it = o.find(okey(r, slot_after(d, r, M)));
    if (it != o.end() && it->second != d.u) return false;
  }
  return true;
}

int window(const std::vector<Dm>& D, const std::vector<int>& live, int r) {
  int r_end = r + 1;
  for (int i : live) r_end = std::max(r_end, D[i].hb + 1);
  int best = 1;
  size_t single = 0;
  for (int w = 1; r + w <= r_end; ++w) {
    const int rr = r + w - 1;
    std::set<int64_t> one, merged;
    for (int i : live) {
      if (D[i].hb >= rr) {
        int64_t a = amount(D[i], rr, 1);
        if (a) one.insert(a);
      }
      int64_t b = amount(D[i], r, w);
      if (b) merged.insert(b);
    }
    single += one.size();
    if (merged.size() <= single) best = w;
  }
  return best;
}

}  // namespace

void build_radix2(const std::vector<int32_t>& pi, const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                  const std::vector<double>& val, int M_, int B, bool wrap, double theta, R2Program& out) {
  const int64_t M = M_;
  const int n = (int)pi.size();
  out = R2Program();
  // demands, self terms
  std::vector<std::pair<int32_t, double>> self;
  std::vector<std::vector<Dm>> per_row(n);
  for (int v = 0; v < n; ++v) {
    for (int e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int u = col[e];
      int64_t d = (int64_t)pi[u] - pi[v];
      if (wrap) {
        d = mod_pos(d, M);
        if (d > M / 2) d -= M;
      }
      if (d == 0) {
        self.push_back({pi[v], val[e]});
        continue;
      }
      Dm x;
      x.u = u;
      x.v = v;
      x.s = pi[u];
      x.e = pi[v];
      x.delta = d;
      x.mag = d < 0 ? -d : d;
      x.sign = d < 0 ? -1 : 1;
      x.hb = 63 - __builtin_clzll((unsigned long long)x.mag);
      x.a = val[e];
      per_row[v].push_back(x);
    }
    std::sort(per_row[v].begin(), per_row[v].end(),
              [](const Dm& a, const Dm& b) { return a.mag != b.mag ? a.mag < b.mag : a.delta < b.delta; });
  }
  std::sort(self.begin(), self.end());
  for (auto& sv : self) {
    out.self.slot.push_back(sv.first);
    out.self.val.push_back(sv.second);
  }
  std::vector<Dm> D;
  size_t kmax = 0;
  for (auto& r : per_row) kmax = std::max(kmax, r.size());
  for (size_t k = 0; k < kmax; ++k)
    for (int v = 0; v < n; ++v)
      if (k < per_row[v].size()) D.push_back(per_row[v][k]);
  // first-fit lanes
  std::vector<Lane> lanes;
  for (int i = 0; i < (int)D.size(); ++i) {
    bool placed = false;
    for (auto& ln : lanes)
      if (fits(ln.occ, D[i], 0, M)) {
        ln.dm.push_back(i);
        occupy(ln.occ, D[i], M);
        placed = true;
        break;
      }
    if (!placed) {
      lanes.emplace_back();
      lanes.back().dm.push_back(i);
      occupy(lanes.back().occ, D[i], M);
    }
  }
  out.n_lanes = (int)lanes.size();
  int R = 0;
  for (auto& d : D) R = std::max(R, d.hb + 1);
  out.reg_depth.push_back(0);
  int out_depth = 1;
  for (int r = 0; r < R; ++r) {
    std::vector<int> at;
    for (int k = 0; k < (int)lanes.size(); ++k) {
      if (lanes[k].bnd != r) continue;
      bool live = false;
      for (int i : lanes[k].dm) live |= D[i].hb >= r;
      if (live) at.push_back(k);
    }
    if (at.empty()) continue;
    std::map<int, std::vector<int>> stepping;     // demands whose values sit in the lane's register
    std::map<int, bool> sparse;
    std::map<int, std::unordered_map<int, int>> home;   // demand -> lane that carries it on (travelling past r)
    for (int k : at) {
      auto& st = stepping[k];
      std::set<int64_t> slots;
      for (int i : lanes[k].dm)
        if (D[i].hb >= r) {
          st.push_back(i);
          slots.insert(slot_after(D[i], r - 1, M));
        }
      sparse[k] = theta > 0 && (double)slots.size() < theta * B;
      for (int i : st)
        if (D[i].hb > r) home[k][i] = k;
    }
    // (a) moves out of sparse lanes
    for (int j : at) {
      if (!sparse[j]) continue;
      std::map<int64_t, std::vector<int>> slots;   // slot after round r -> demands
      for (int i : stepping[j])
        if (D[i].hb > r) slots[slot_after(D[i], r, M)].push_back(i);
      for (int ii : at) {
        if (ii >= j || slots.empty()) break;
        if (sparse[ii] || lanes[ii].depth != lanes[j].depth) continue;
        bool steps = false;
        for (int i : stepping[ii]) steps |= ((D[i].mag >> r) & 1) != 0;
        if (!steps) continue;
        Occ& oi = lanes[ii].occ;
        for (auto it = slots.begin(); it != slots.end();) {
          const auto& ds = it->second;
          if (oi.count(okey(r, it->first))) {
            ++it;
            continue;
          }
          bool ok = true;
          for (int i : ds) ok = ok && fits(oi, D[i], r + 1, M);
          if (!ok) {
            ++it;
            continue;
          }
          oi[okey(r, it->first)] = D[ds[0]].u;
          for (int i : ds) {
            for (int x = r + 1; x < D[i].hb; ++x) oi[okey(x, slot_after(D[i], x, M))] = D[i].u;
            home[j][i] = ii;
            lanes[ii].dm.push_back(i);
            ++out.n_moved;
          }
          it = slots.erase(it);
        }
      }
      bool any = false;
      for (auto& kv : home[j]) any |= kv.second != j;
      if (any) {
        std::vector<int> keep;
        for (int i : lanes[j].dm) {
          auto h = home[j].find(i);
          if (h == home[j].end() || h->second == j) keep.push_back(i);
        }
        lanes[j].dm = keep;
        lanes[j].occ.clear();
        for (int i : keep) occupy(lanes[j].occ, D[i], M);
      }
    }
    // (b) windows of what sparse lanes keep
    std::map<int, int> win;
    auto own = [&](int k, int i) { return D[i].hb == r || home[k].at(i) == k; };
    for (int k : at) {
      std::vector<int> mine;
      for (int i : stepping[k])
        if (own(k, i)) mine.push_back(i);
      win[k] = (sparse[k] && !mine.empty()) ? window(D, mine, r) : 1;
    }
    // lanes in which nothing moves skip the round
    std::set<int> idle;
    for (int k : at) {
      bool moves = false;
      for (auto& kv : home[k]) moves |= kv.second != k;
      for (int i : stepping[k]) moves |= amount(D[i], r, win[k]) != 0;
      if (!moves) idle.insert(k);
    }
    // next registers, lanes in creation order
    std::set<int> receives;
    for (int k : at)
      for (int i : stepping[k]) {
        if (D[i].hb <= r) continue;
        const int h = home[k].at(i);
        if (h != k || D[i].hb >= r + win[k]) receives.insert(h);
      }
    std::map<int, int> dst;
    for (int k : at)
      if (receives.count(k) && !idle.count(k)) {
        dst[k] = (int)out.reg_depth.size();
        out.reg_depth.push_back(lanes[k].depth + 1);
      }
    for (int k : at) {
      if (idle.count(k)) continue;
      const Lane& ln = lanes[k];
      std::map<std::pair<int, int64_t>, std::map<int64_t, double>> keep;
      std::map<int64_t, std::map<int64_t, double>> fin;
      for (int i : stepping[k]) {
        const Dm& d = D[i];
        const int wd = own(k, i) ? win[k] : 1;      // moved demands take one round
        const int64_t m = amount(d, r, wd);
        if (d.hb < r + wd) {
          fin[m][d.e] = d.a;
          continue;
        }
        const int tgt = dst.at(home[k].at(i));
        keep[{tgt, m}][slot_after(d, r + wd - 1, M)] = 1.0;   // one source per slot: shared entries coincide
      }
      R2Step st;
      st.lane = k;
      st.r0 = r;
      st.r1 = r + win[k];
      st.depth = ln.depth;
      st.src = ln.reg;
      for (auto& kv : keep) {
        R2Term t;
        t.dst = kv.first.first;
        t.m = kv.first.second;
        for (auto& sv : kv.second) {
          t.slot.push_back((int32_t)sv.first);
          t.val.push_back(sv.second);
        }
        st.keep.push_back(std::move(t));
      }
      for (auto& kv : fin) {
        R2Term t;
        t.m = kv.first;
        for (auto& sv : kv.second) {
          t.slot.push_back((int32_t)sv.first);
          t.val.push_back(sv.second);
        }
        st.fin.push_back(std::move(t));
      }
      out.steps.push_back(std::move(st));
      out_depth = std::max(out_depth, ln.depth + 1);
    }
    for (int k : at) {
      Lane& ln = lanes[k];
      ln.bnd = r + win[k];
      if (!idle.count(k)) {
        ln.depth += 1;
        auto it = dst.find(k);
        ln.reg = it == dst.end() ? -1 : it->second;
      }
    }
  }
  out.depth = out_depth;
  out.ops.push_back({-1, 0, 0});
  for (int s = 0; s < (int)out.steps.size(); ++s) {
    const R2Step& st = out.steps[s];
    for (int t = 0; t < (int)(st.keep.size() + st.fin.size()); ++t) out.ops.push_back({s, t, st.depth});
  }
}

}  // namespace ficgcn
