// Batched hybrid key switching and batched ciphertext kernels.
//
// A batch holds R key switches at one level whose inputs come from U
// distinct source polynomials (U = 1 when every rotation of one ciphertext
// is hoisted on its ModUp; U = R when each ciphertext is switched once, as
// for relinearising a layer).  Each stage is one launch over the batch:
//   ModUp  : inverse NTT of the U sources, fast base conversion of every
//            digit of every source, forward NTT of the extended limbs;
//   inner  : acc_r = sum_d sigma_{g_r}(D_{src(r),d}) * key_{r,d}   (both components);
//   ModDown: inverse NTT of the P limbs of every acc_r, rounded conversion
//            to Q_l, forward NTT, then the grouped final step
//            out_grp (+)= sum_r ((acc_r - conv_r) * P^-1 + add_r) [(.) pt_r].
// Every switch is the same exact modular computation as a single key
// switch (ModUp, automorphism on the digits, inner product, ModDown with
// rounding), so the words equal those of R separate switches.  The
// grouped final step replaces "write R switched ciphertexts, read them
// back for a masked sum" by one read of acc and conv per switch.
#include <algorithm>
#include <numeric>

#include "internal.h"
#include "fpmod.h"
#include "ks_batch.h"

namespace ficgcn {

void zero_fill(ckks_ctx* c, uint64_t* p, size_t words);

constexpr int KB = 256;

// Accesses through pointers read from device tables (job lists, term lists,
// pointer arrays).  The compiler cannot tell that such a pointer addresses
// global memory and would emit flat accesses, which also count on the
// scalar-load counter: every read of the next table entry would then wait for
// all vector loads in flight.  These pin the access to the global segment.
typedef __attribute__((address_space(1))) uint64_t gu64;
__device__ __forceinline__ uint64_t gld(const uint64_t* p) { return *(const gu64*)p; }
__device__ __forceinline__ void gst(uint64_t* p, uint64_t v) { *(gu64*)p = v; }
__device__ const uint64_t k_one_word = 1;

__device__ __forceinline__ uint32_t auto_idx(uint32_t k, uint64_t g, int log_n) {
  // evaluation index k holds A(psi^(2 brev(k) + 1)); sigma_g reads the index of psi^(g (2 brev(k) + 1))
  uint32_t N2 = 2u << log_n;
  uint32_t e = 2u * bitrev(k, log_n) + 1u;
  uint32_t ge = (uint32_t)(((uint64_t)e * g) & (N2 - 1));
  return bitrev((ge - 1u) >> 1, log_n);
}

// tmp[u] = sources[u] (l1 limbs)
__global__ void k_gather(uint64_t* __restrict__ tmp, const uint64_t* const* __restrict__ src, int l1, int log_n) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int i = blockIdx.y, u = blockIdx.z;
  tmp[((size_t)u * l1 + i) * N + j] = gld(src[u] + (size_t)i * N + j);
}

struct DigitTables {
  enum { MAX = 32 };
  const uint64_t* tab[MAX];   // [n_src] hat_inv, [n_src] Shoup, [n_dst][n_src] hat mod dst
  const int* idx[MAX];        // [n_src] source moduli, then [n_dst] destination moduli
  int n_src[MAX];
  int n_dst[MAX];
};

// Digit d of source u: the digit's residues (coefficient form, in tmp)
// converted to every other prime of Q_l and P; the digit's own limbs are
// the source limbs in evaluation form.
__global__ void k_modup_conv(const uint64_t* __restrict__ tmp, const uint64_t* const* __restrict__ src,
                             uint64_t* __restrict__ D, DigitTables dt, int alpha, int l1, int ext, int nd, int L,
                             int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int d = blockIdx.y, u = blockIdx.z;
  const uint64_t* tab = dt.tab[d];
  const int* idx = dt.idx[d];
  const int ns = dt.n_src[d], ndst = dt.n_dst[d];
  const uint64_t* s = tmp + ((size_t)u * l1 + (size_t)d * alpha) * N;
  const uint64_t* own = src[u] + (size_t)d * alpha * N;
  uint64_t* Dd = D + ((size_t)u * nd + d) * ext * N;
  uint64_t y[8];
  for (int t = 0; t < ns; ++t) {
    const uint64_t b = mods[idx[t]].q;
    y[t] = mul_shoup(s[t * N + j], tab[t], tab[ns + t], b);
    Dd[((size_t)d * alpha + t) * N + j] = gld(own + t * N + j);
  }
  const uint64_t* hm = tab + 2 * ns;
  for (int k = 0; k < ndst; ++k) {
    const int m = idx[ns + k];
    const Mod md = mods[m];
    u128 acc = 0;
    for (int t = 0; t < ns; ++t) acc += (u128)y[t] * hm[k * ns + t];
    const int pos = m < L ? m : m - L + l1;
    Dd[(size_t)pos * N + j] = reduce128(acc, md);
  }
}

// acc[r][c][i] = sum_d D_{src(r),d}[i][sigma_g(j)] * key_r[d][c][m(i)][j]
__global__ void k_keymac_batch(uint64_t* __restrict__ acc, const uint64_t* __restrict__ D,
                               const KSJob* __restrict__ jobs, int nd, int ext, int l1, int L, int n_mod, int log_n,
                               const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * KB + threadIdx.x;
  const int i = blockIdx.y, r = blockIdx.z;
  const KSJob jb = jobs[r];
  const int m = i < l1 ? i : i - l1 + L;
  const uint32_t jj = jb.g == 1 ? j : auto_idx(j, jb.g, log_n);
  const uint64_t* Du = D + (size_t)jb.src * nd * ext * N;
  u128 s0 = 0, s1 = 0;
  for (int d = 0; d < nd; ++d) {
    const u128 x = Du[((size_t)d * ext + i) * N + jj];
    s0 += x * gld(jb.key + (((size_t)d * 2 + 0) * n_mod + m) * N + j);
    s1 += x * gld(jb.key + (((size_t)d * 2 + 1) * n_mod + m) * N + j);
  }
  const Mod md = mods[m];
  acc[(((size_t)r * 2 + 0) * ext + i) * N + j] = reduce128(s0, md);
  acc[(((size_t)r * 2 + 1) * ext + i) * N + j] = reduce128(s1, md);
}

// The same inner products with jobs taken in runs that share one key (and Galois element):
// a thread reads its key words once and applies them to every job of its run (the rotations
// of several ciphertexts by one step), so the key streams from HBM once per run.
constexpr int KR_MAXD = 8;   // digits held in registers (the kernels are instantiated per digit count)
template <int ND>
__global__ void k_keymac_runs(uint64_t* __restrict__ acc, const uint64_t* __restrict__ D,
                              const KSJob* __restrict__ jobs, const int* __restrict__ run_start, int ext, int l1,
                              int L, int n_mod, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * KB + threadIdx.x;
  const int i = blockIdx.y;
  const int r0 = run_start[blockIdx.z], r1 = run_start[blockIdx.z + 1];
  const KSJob j0 = jobs[r0];
  const int m = i < l1 ? i : i - l1 + L;
  const uint32_t jj = j0.g == 1 ? j : auto_idx(j, j0.g, log_n);
  uint64_t k0[ND], k1[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    k0[d] = gld(j0.key + (((size_t)d * 2 + 0) * n_mod + m) * N + j);
    k1[d] = gld(j0.key + (((size_t)d * 2 + 1) * n_mod + m) * N + j);
  }
  const Mod md = mods[m];
  for (int r = r0; r < r1; ++r) {
    const uint64_t* Du = D + (size_t)jobs[r].src * ND * ext * N;
    u128 s0 = 0, s1 = 0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const u128 x = Du[((size_t)d * ext + i) * N + jj];
      s0 += x * k0[d];
      s1 += x * k1[d];
    }
    acc[(((size_t)r * 2 + 0) * ext + i) * N + j] = reduce128(s0, md);
    acc[(((size_t)r * 2 + 1) * ext + i) * N + j] = reduce128(s1, md);
  }
}

// runs of consecutive jobs with one key and Galois element; host side
static std::vector<int> key_runs(const std::vector<KSJob>& jobs) {
  std::vector<int> start;
  for (size_t r = 0; r < jobs.size(); ++r)
    if (r == 0 || jobs[r].key != jobs[r - 1].key || jobs[r].g != jobs[r - 1].g) start.push_back((int)r);
  start.push_back((int)jobs.size());
  return start;
}

struct MDK {
  uint64_t hP[8];                 // floor(P/2) mod p_t
  uint64_t hQ[64];                // floor(P/2) mod q_i
  uint64_t pinv[64], pinv_s[64];  // P^-1 mod q_i, Shoup
};

// conv[z][i] = FastBConv_{P -> q_i}([acc_P + floor(P/2)]) - floor(P/2)   (coefficient form)
__global__ void k_moddown_conv_batch(const uint64_t* __restrict__ acc, int ext, int l1, const int* __restrict__ src_mod,
                                     const int* __restrict__ dst_mod, int ns, const uint64_t* __restrict__ table,
                                     MDK k, uint64_t* __restrict__ conv, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int z = blockIdx.y;   // r * 2 + component
  const uint64_t* ap = acc + ((size_t)z * ext + l1) * N;
  uint64_t y[8];
  for (int t = 0; t < ns; ++t) {
    const uint64_t b = mods[src_mod[t]].q;
    const uint64_t x = add_mod(ap[t * N + j], k.hP[t], b);
    y[t] = mul_shoup(x, table[t], table[ns + t], b);
  }
  const uint64_t* hm = table + 2 * ns;
  for (int d = 0; d < l1; ++d) {
    const Mod md = mods[dst_mod[d]];
    u128 a = 0;
    for (int t = 0; t < ns; ++t) a += (u128)y[t] * hm[d * ns + t];
    conv[((size_t)z * l1 + d) * N + j] = sub_mod(reduce128(a, md), k.hQ[d], md.q);
  }
}

struct GroupDesc {
  uint64_t* out;   // [2][l+1][N]
  int start, end;  // job range within the chunk
  int accumulate;
  int pad;
};

__global__ void k_ks_final(const uint64_t* __restrict__ acc, const uint64_t* __restrict__ conv, int ext, int l1, MDK k,
                           const KSJob* __restrict__ jobs, const GroupDesc* __restrict__ groups, int log_n,
                           const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * KB + threadIdx.x;
  const int i = blockIdx.y;
  const int comp = blockIdx.z & 1;
  const GroupDesc gd = groups[blockIdx.z >> 1];
  const Mod md = mods[i];
  const uint64_t q = md.q;
  const size_t o = ((size_t)comp * l1 + i) * N + j;
  uint64_t a = gd.accumulate ? gld(gd.out + o) : 0;
  u128 s = 0;
  int cnt = 0;
  for (int r = gd.start; r < gd.end; ++r) {
    const KSJob jb = jobs[r];
    uint64_t v = sub_mod(acc[(((size_t)r * 2 + comp) * ext + i) * N + j],
                         conv[(((size_t)r * 2 + comp) * l1 + i) * N + j], q);
    v = mul_shoup(v, k.pinv[i], k.pinv_s[i], q);
    if (comp == 0 && jb.add0) v = add_mod(v, gld(jb.add0 + (size_t)i * N + (jb.g == 1 ? j : auto_idx(j, jb.g, log_n))), q);
    if (comp == 1 && jb.add1) v = add_mod(v, gld(jb.add1 + (size_t)i * N + j), q);
    if (jb.pt) {
      s += (u128)v * gld(jb.pt + (size_t)i * N + j);
      if (++cnt == 8) {
        a = add_mod(a, reduce128(s, md), q);
        s = 0;
        cnt = 0;
      }
    } else {
      a = add_mod(a, v, q);
    }
  }
  gst(gd.out + o, add_mod(a, reduce128(s, md), q));
}

static MDK mdk(ckks_ctx* c, int level) {
  MDK k{};
  for (int t = 0; t < c->alpha; ++t) {
    const uint64_t pm = c->mod[c->L + t];
    uint64_t P_mod = 1;
    for (int u = 0; u < c->alpha; ++u) P_mod = (uint64_t)((u128)P_mod * (c->mod[c->L + u] % pm) % pm);
    k.hP[t] = (uint64_t)((u128)sub_mod(P_mod, 1, pm) * invmod(2, pm) % pm);
  }
  for (int i = 0; i <= level; ++i) {
    const uint64_t q = c->mod[i];
    uint64_t P_mod = 1;
    for (int u = 0; u < c->alpha; ++u) P_mod = (uint64_t)((u128)P_mod * (c->mod[c->L + u] % q) % q);
    k.hQ[i] = (uint64_t)((u128)sub_mod(P_mod, 1, q) * invmod(2, q) % q);
    k.pinv[i] = invmod(P_mod, q);
    k.pinv_s[i] = shoup(k.pinv[i], q);
  }
  return k;
}

enum { S_KB_TMP = 50, S_KB_D, S_KB_ACC, S_KB_CONV, S_KB_JOBS, S_KB_SRC, S_KB_GRP, S_TB_JOBS, S_RS_PTR, S_RS_LAST,
       S_RS_D, S_GM_TERMS, S_GM_START, S_GM_OUT, S_KB_RUNS };

template <typename T>
static T* upload(ckks_ctx* c, int slot, const std::vector<T>& v) {
  return (T*)dev_table(c, slot, v.data(), v.size() * sizeof(T));
}

// scratch bound of one chunk of a key-switch batch
static constexpr size_t KS_BUDGET = (size_t)3 << 30;

void keyswitch_batch(ckks_ctx* c, int level, const std::vector<const uint64_t*>& sources,
                     const std::vector<KSJob>& jobs, const std::vector<uint64_t*>& outs, bool accumulate) {
  const size_t N = c->N;
  const int l1 = level + 1, ext = l1 + c->alpha;
  const int nd = (l1 + c->alpha - 1) / c->alpha;
  const int n_grp = (int)outs.size();
  if (c->alpha > 8 || l1 > 64 || nd > DigitTables::MAX) FICGCN_THROW(EINVAL_, "too many primes");
  for (size_t r = 0; r < jobs.size(); ++r) {
    const KSJob& jb = jobs[r];
    if (jb.src < 0 || jb.src >= (int)sources.size() || !sources[jb.src] || !jb.key || jb.grp < 0 || jb.grp >= n_grp ||
        !outs[jb.grp] || (r && jobs[r - 1].grp > jb.grp))
      FICGCN_THROW(EINVAL_, "bad key-switch job");
  }
  ProfScope ps(c, "ks_batch");
  const size_t per_job = (size_t)2 * (ext + l1) * N * 8;
  const size_t per_src = (size_t)(nd * ext + l1) * N * 8;
  std::vector<char> touched(n_grp, 0);
  const MDK k = mdk(c, level);
  DigitTables dt{};
  for (int d = 0; d < nd; ++d) {
    const BConv& bc = get_modup(c, level, d);
    dt.tab[d] = bc.dev;
    dt.idx[d] = bc.idx;
    dt.n_src[d] = bc.n_src;
    dt.n_dst[d] = bc.n_dst;
  }
  const BConv& md = get_moddown(c, level);
  size_t a = 0;
  while (a < jobs.size()) {
    // chunk [a, b): sources remapped to a dense local list
    std::vector<int> local(sources.size(), -1);
    std::vector<const uint64_t*> srcs;
    std::vector<KSJob> cj;
    size_t b = a, bytes = 0;
    while (b < jobs.size()) {
      const bool new_src = local[jobs[b].src] < 0;
      const size_t add = per_job + (new_src ? per_src : 0);
      if (b > a && bytes + add > KS_BUDGET) break;
      bytes += add;
      if (new_src) {
        local[jobs[b].src] = (int)srcs.size();
        srcs.push_back(sources[jobs[b].src]);
      }
      KSJob j = jobs[b];
      j.src = local[j.src];
      cj.push_back(j);
      ++b;
    }
    // groups of the chunk (contiguous since jobs are sorted by group)
    std::vector<GroupDesc> gds;
    for (size_t r = 0; r < cj.size(); ++r) {
      const int g = cj[r].grp;
      if (gds.empty() || r == 0 || cj[r - 1].grp != g) {
        gds.push_back(GroupDesc{outs[g], (int)r, (int)r + 1, (accumulate || touched[g]) ? 1 : 0, 0});
        touched[g] = 1;
      } else {
        gds.back().end = (int)r + 1;
      }
    }
    const int U = (int)srcs.size(), R = (int)cj.size();
    KSJob* jd = upload(c, S_KB_JOBS, cj);
    const uint64_t* const* sd = upload(c, S_KB_SRC, srcs);
    GroupDesc* gd = upload(c, S_KB_GRP, gds);
    uint64_t* tmp = (uint64_t*)dev_scratch(c, S_KB_TMP, (size_t)U * l1 * N * 8);
    uint64_t* D = (uint64_t*)dev_scratch(c, S_KB_D, (size_t)U * nd * ext * N * 8);
    uint64_t* acc = (uint64_t*)dev_scratch(c, S_KB_ACC, (size_t)R * 2 * ext * N * 8);
    uint64_t* conv = (uint64_t*)dev_scratch(c, S_KB_CONV, (size_t)R * 2 * l1 * N * 8);
    {
      ProfScope pm(c, "modup");
      hipLaunchKernelGGL(k_gather, dim3(N / KB, l1, U), dim3(KB), 0, c->stream, tmp, sd, l1, c->log_n);
      HIPCHECK(hipGetLastError());
      ntt_inv(c, tmp, l1, lm_q(l1), U, (size_t)l1 * N);
      hipLaunchKernelGGL(k_modup_conv, dim3(N / KB, nd, U), dim3(KB), 0, c->stream, tmp, sd, D, dt, c->alpha, l1, ext,
                         nd, c->L, c->log_n, c->t.mods);
      HIPCHECK(hipGetLastError());
      // every extended limb to evaluation form except each digit's own limbs
      ntt_fwd(c, D, ext, lm_ext(level, c->L), U * nd, (size_t)ext * N, c->alpha, l1);
    }
    {
      ProfScope pk(c, "keymac");
      const std::vector<int> runs = key_runs(cj);
      const int n_runs = (int)runs.size() - 1;
      if (n_runs < R && nd <= KR_MAXD) {   // some jobs share a key: each key read once per run
        const int* rd = upload(c, S_KB_RUNS, runs);
        const dim3 grid(N / KB, ext, n_runs);
#define KR_LAUNCH(NDV)                                                                                          \
  hipLaunchKernelGGL(k_keymac_runs<NDV>, grid, dim3(KB), 0, c->stream, acc, D, jd, rd, ext, l1, c->L, c->n_mod(), \
                     c->log_n, c->t.mods)
        switch (nd) {
          case 1: KR_LAUNCH(1); break;
          case 2: KR_LAUNCH(2); break;
          case 3: KR_LAUNCH(3); break;
          case 4: KR_LAUNCH(4); break;
          case 5: KR_LAUNCH(5); break;
          case 6: KR_LAUNCH(6); break;
          case 7: KR_LAUNCH(7); break;
          default: KR_LAUNCH(8);
        }
#undef KR_LAUNCH
      } else {
        hipLaunchKernelGGL(k_keymac_batch, dim3(N / KB, ext, R), dim3(KB), 0, c->stream, acc, D, jd, nd, ext, l1,
                           c->L, c->n_mod(), c->log_n, c->t.mods);
      }
      HIPCHECK(hipGetLastError());
    }
    {
      ProfScope pd(c, "moddown");
      ntt_inv(c, acc + (size_t)l1 * N, c->alpha, LimbMap{c->L, 1 << 30, 0}, 2 * R, (size_t)ext * N);
      hipLaunchKernelGGL(k_moddown_conv_batch, dim3(N / KB, 2 * R), dim3(KB), 0, c->stream, acc, ext, l1, md.idx,
                         md.idx + md.n_src, md.n_src, (const uint64_t*)md.dev, k, conv, c->log_n, c->t.mods);
      HIPCHECK(hipGetLastError());
      ntt_fwd(c, conv, l1, lm_q(l1), 2 * R, (size_t)l1 * N);
      hipLaunchKernelGGL(k_ks_final, dim3(N / KB, l1, 2 * gds.size()), dim3(KB), 0, c->stream, acc, conv, ext, l1, k,
                         jd, gd, c->log_n, c->t.mods);
      HIPCHECK(hipGetLastError());
    }
    // the host lists of this chunk are released below and the device lists reused
    stream_sync(c);
    a = b;
  }
  if (!accumulate)
    for (int g = 0; g < n_grp; ++g)
      if (!touched[g]) zero_fill(c, outs[g], (size_t)2 * l1 * N);
}

// ---- masked sums of key switches before one ModDown (double hoisting) ---------

struct MaskGroup {
  int start, end;   // job range (all jobs of the batch, sorted by group)
};

// The key inner products of a group's jobs and their masked sum in one pass:
// per job r, acc_r[c][i] = sum_d D_{src(r),d}[i][sigma_g(j)] * key_r[d][c][m(i)][j]
// (reduced), then A[c][i] += acc_r[c][i] (.) pt_r[i] (or + acc_r without a
// mask), both components per thread.  acc_r is never stored: the sums are
// those of the batched key inner product followed by a masked sum of its
// outputs, in the same order.
__global__ void k_keymac_masked(const uint64_t* __restrict__ D, const KSJob* __restrict__ jobs,
                                const GroupDesc* __restrict__ groups, int nd, int ext, int l1, int L, int n_mod,
                                int log_n, int n_groups, int xcd_order, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  // xcd_order: the groups of one coefficient block run back to back on one XCD
  // (blocks go round-robin over the 8 XCDs by linear id), so the keys the
  // groups share (one per shift) are read into that XCD's L2 once
  int jb, gi;
  if (xcd_order) {
    const int b = blockIdx.x, idx = b >> 3;
    jb = (b & 7) + 8 * (idx / n_groups);
    gi = idx % n_groups;
  } else {
    jb = blockIdx.x;
    gi = blockIdx.z;
  }
  const uint32_t j = (uint32_t)jb * KB + threadIdx.x;
  const int i = blockIdx.y;
  const GroupDesc gd = groups[gi];
  const int m = i < l1 ? i : i - l1 + L;
  const Mod md = mods[m];
  uint64_t* a0 = gd.out + (size_t)i * N + j;              // gd.out: this group's A
  uint64_t* a1 = gd.out + ((size_t)ext + i) * N + j;
  uint64_t v0 = gld(a0), v1 = gld(a1);
  u128 t0 = 0, t1 = 0;
  int cnt = 0;
  for (int r = gd.start; r < gd.end; ++r) {
    const KSJob jb = jobs[r];
    const uint32_t jj = jb.g == 1 ? j : auto_idx(j, jb.g, log_n);
    const uint64_t* Du = D + (size_t)jb.src * nd * ext * N;
    u128 s0 = 0, s1 = 0;
    for (int d = 0; d < nd; ++d) {
      const u128 x = Du[((size_t)d * ext + i) * N + jj];
      s0 += x * gld(jb.key + (((size_t)d * 2 + 0) * n_mod + m) * N + j);
      s1 += x * gld(jb.key + (((size_t)d * 2 + 1) * n_mod + m) * N + j);
    }
    const uint64_t x0 = reduce128(s0, md), x1 = reduce128(s1, md);
    if (jb.pt) {
      const uint64_t p = gld(jb.pt + (size_t)i * N + j);
      t0 += (u128)x0 * p;
      t1 += (u128)x1 * p;
    } else {
      t0 += x0;
      t1 += x1;
    }
    if (++cnt == 8) {
      v0 = add_mod(v0, reduce128(t0, md), md.q);
      v1 = add_mod(v1, reduce128(t1, md), md.q);
      t0 = 0;
      t1 = 0;
      cnt = 0;
    }
  }
  gst(a0, add_mod(v0, reduce128(t0, md), md.q));
  gst(a1, add_mod(v1, reduce128(t1, md), md.q));
}

// The masked key inner products of a chunk with its jobs taken key by key (runs of jobs
// sharing one key and Galois element, at most KM_MAXG output groups): a thread per (coefficient,
// limb) reads each key word once for its run and adds every job's product, times its
// plaintext, to its group's sum.  The runs are split in n_seg segments (blockIdx.z) whose sums
// go to P[seg][group][component] and are added to the accumulators by k_masked_combine.
// Limbs of Q primes in (2^49, 2^50) (fq): the products in fp64 residues (fpmod.h), each an
// exact signed representative in (-q, q); a job's digit sum is brought back before its mask
// product, and the group sums every four jobs, so every double stays an exact integer below
// 2^53.  The words equal those of the integer form, which the special primes' limbs take.
constexpr int KM_MAXG = 4;
template <int ND, int NG>
__global__ void k_keymac_masked_runs(const uint64_t* __restrict__ D, const KSJob* __restrict__ jobs,
                                     const int* __restrict__ run_start, int n_runs, int n_seg,
                                     const int* __restrict__ job_gl, int n_gl, uint64_t* __restrict__ P, int ext,
                                     int l1, int L, int n_mod, int log_n, int fq, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * KB + threadIdx.x;
  const int i = blockIdx.y, seg = blockIdx.z;
  const int m = i < l1 ? i : i - l1 + L;
  const Mod md = mods[m];
  const int ra = (int)((int64_t)n_runs * seg / n_seg), rb = (int)((int64_t)n_runs * (seg + 1) / n_seg);
  if (fq && i < l1) {
    const double qd = (double)md.q, qinv = 1.0 / qd;
    auto cv = [](uint64_t v) { return b2f(to_fbits(v)); };
    double T0[NG], T1[NG];
    int cnt[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      T0[g] = T1[g] = 0.0;
      cnt[g] = 0;
    }
    for (int run = ra; run < rb; ++run) {
      const int r0 = run_start[run], r1 = run_start[run + 1];
      const KSJob j0 = jobs[r0];
      const uint32_t jj = j0.g == 1 ? j : auto_idx(j, j0.g, log_n);
      double k0[ND], k1[ND];
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        k0[d] = cv(gld(j0.key + (((size_t)d * 2 + 0) * n_mod + m) * N + j));
        k1[d] = cv(gld(j0.key + (((size_t)d * 2 + 1) * n_mod + m) * N + j));
      }
      for (int r = r0; r < r1; ++r) {
        const KSJob jb = jobs[r];
        const uint64_t* Du = D + (size_t)jb.src * ND * ext * N;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const double x = cv(Du[((size_t)d * ext + i) * N + jj]);
          s0 += fmulmod_s(x, k0[d], qd, qinv);
          s1 += fmulmod_s(x, k1[d], qd, qinv);
        }
        s0 = sred(s0, qd, qinv);
        s1 = sred(s1, qd, qinv);
        if (jb.pt) {   // one job per thread block step: no divergence
          const double p = cv(gld(jb.pt + (size_t)i * N + j));
          s0 = fmulmod_s(s0, p, qd, qinv);
          s1 = fmulmod_s(s1, p, qd, qinv);
        }
        const int gl = job_gl[r];
#pragma unroll
        for (int g = 0; g < NG; ++g)
          if (g == gl) {
            T0[g] += s0;
            T1[g] += s1;
            if (++cnt[g] == 4) {
              T0[g] = sred(T0[g], qd, qinv);
              T1[g] = sred(T1[g], qd, qinv);
              cnt[g] = 0;
            }
          }
      }
    }
#pragma unroll
    for (int g = 0; g < NG; ++g)
      if (g < n_gl) {
        P[((((size_t)seg * n_gl + g) * 2 + 0) * ext + i) * N + j] = from_fbits(f2b(canon(sred(T0[g], qd, qinv), qd)));
        P[((((size_t)seg * n_gl + g) * 2 + 1) * ext + i) * N + j] = from_fbits(f2b(canon(sred(T1[g], qd, qinv), qd)));
      }
    return;
  }
  u128 t0[NG], t1[NG];
  uint64_t v0[NG], v1[NG];
  int cnt[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    t0[g] = t1[g] = 0;
    v0[g] = v1[g] = 0;
    cnt[g] = 0;
  }
  for (int run = ra; run < rb; ++run) {
    const int r0 = run_start[run], r1 = run_start[run + 1];
    const KSJob j0 = jobs[r0];
    const uint32_t jj = j0.g == 1 ? j : auto_idx(j, j0.g, log_n);
    uint64_t k0[ND], k1[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      k0[d] = gld(j0.key + (((size_t)d * 2 + 0) * n_mod + m) * N + j);
      k1[d] = gld(j0.key + (((size_t)d * 2 + 1) * n_mod + m) * N + j);
    }
    for (int r = r0; r < r1; ++r) {
      const KSJob jb = jobs[r];
      const uint64_t* Du = D + (size_t)jb.src * ND * ext * N;
      u128 s0 = 0, s1 = 0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        const u128 x = Du[((size_t)d * ext + i) * N + jj];
        s0 += x * k0[d];
        s1 += x * k1[d];
      }
      const uint64_t x0 = reduce128(s0, md), x1 = reduce128(s1, md);
      u128 y0 = x0, y1 = x1;
      if (jb.pt) {   // one job per thread block step: no divergence
        const uint64_t p = gld(jb.pt + (size_t)i * N + j);
        y0 = (u128)x0 * p;
        y1 = (u128)x1 * p;
      }
      const int gl = job_gl[r];
#pragma unroll
      for (int g = 0; g < NG; ++g)
        if (g == gl) {
          t0[g] += y0;
          t1[g] += y1;
          if (++cnt[g] == 8) {
            v0[g] = add_mod(v0[g], reduce128(t0[g], md), md.q);
            v1[g] = add_mod(v1[g], reduce128(t1[g], md), md.q);
            t0[g] = t1[g] = 0;
            cnt[g] = 0;
          }
        }
    }
  }
#pragma unroll
  for (int g = 0; g < NG; ++g)
    if (g < n_gl) {
      P[((((size_t)seg * n_gl + g) * 2 + 0) * ext + i) * N + j] = add_mod(v0[g], reduce128(t0[g], md), md.q);
      P[((((size_t)seg * n_gl + g) * 2 + 1) * ext + i) * N + j] = add_mod(v1[g], reduce128(t1[g], md), md.q);
    }
}

// A_group += sum over the segments of P[seg][group] (both components, every limb of the key basis)
__global__ void k_masked_combine(const GroupDesc* __restrict__ groups, const uint64_t* __restrict__ P, int n_gl,
                                 int n_seg, int ext, int l1, int L, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * KB + threadIdx.x;
  const int i = blockIdx.y, g = blockIdx.z >> 1, comp = blockIdx.z & 1;
  const int m = i < l1 ? i : i - l1 + L;
  const uint64_t q = mods[m].q;
  uint64_t* a = groups[g].out + ((size_t)comp * ext + i) * N + j;
  uint64_t v = gld(a);
  for (int sg = 0; sg < n_seg; ++sg) v = add_mod(v, P[((((size_t)sg * n_gl + g) * 2 + comp) * ext + i) * N + j], q);
  gst(a, v);
}

// out_grp (+)= (A_Q - conv) P^-1  [+ sum_r sigma_g(add0_r) (.) pt_r on component 0]
__global__ void k_masked_final(const uint64_t* __restrict__ A, const uint64_t* __restrict__ conv, int ext, int l1,
                               MDK k, const KSJob* __restrict__ jobs, const MaskGroup* __restrict__ groups,
                               uint64_t* const* __restrict__ outs, int accumulate, int log_n,
                               const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * KB + threadIdx.x;
  const int i = blockIdx.y;
  const int comp = blockIdx.z & 1, g = blockIdx.z >> 1;
  const Mod md = mods[i];
  const uint64_t q = md.q;
  const size_t o = ((size_t)comp * l1 + i) * N + j;
  uint64_t v = sub_mod(A[(((size_t)g * 2 + comp) * ext + i) * N + j], conv[(((size_t)g * 2 + comp) * l1 + i) * N + j], q);
  v = mul_shoup(v, k.pinv[i], k.pinv_s[i], q);
  if (comp == 0) {
    const MaskGroup gr = groups[g];
    u128 s = 0;
    int cnt = 0;
    for (int r = gr.start; r < gr.end; ++r) {
      const KSJob jb = jobs[r];
      if (!jb.add0) continue;
      const uint64_t x = gld(jb.add0 + (size_t)i * N + (jb.g == 1 ? j : auto_idx(j, jb.g, log_n)));
      s += jb.pt ? (u128)x * gld(jb.pt + (size_t)i * N + j) : (u128)x;
      if (++cnt == 8) {
        v = add_mod(v, reduce128(s, md), q);
        s = 0;
        cnt = 0;
      }
    }
    v = add_mod(v, reduce128(s, md), q);
  }
  uint64_t* out = outs[g];
  gst(out + o, accumulate ? add_mod(gld(out + o), v, q) : v);
}

enum { S_KM_A = 80, S_KM_CONV, S_KM_JOBS, S_KM_GRP, S_KM_OUT, S_KM_CGRP, S_KM_RUNS, S_KM_GL, S_KM_P };

void keyswitch_masked_sum(ckks_ctx* c, int level, const std::vector<const uint64_t*>& sources,
                          const std::vector<KSJob>& jobs, const std::vector<uint64_t*>& outs, bool accumulate) {
  const size_t N = c->N;
  const int l1 = level + 1, ext = l1 + c->alpha;
  const int nd = (l1 + c->alpha - 1) / c->alpha;
  const int n_grp = (int)outs.size();
  if (c->alpha > 8 || l1 > 64 || nd > DigitTables::MAX) FICGCN_THROW(EINVAL_, "too many primes");
  if (n_grp == 0) return;
  for (size_t r = 0; r < jobs.size(); ++r) {
    const KSJob& jb = jobs[r];
    if (jb.src < 0 || jb.src >= (int)sources.size() || !sources[jb.src] || !jb.key || jb.grp < 0 ||
        jb.grp >= n_grp || (r && jobs[r - 1].grp > jb.grp))
      FICGCN_THROW(EINVAL_, "bad masked key-switch job");
  }
  for (uint64_t* o : outs)
    if (!o) FICGCN_THROW(EINVAL_, "null output");
  // at most KM_MAXG outputs: the jobs go key by key (before chunking, so a chunk holds every use
  // of its keys) and every key is read once for all outputs that use it
  const bool by_key = n_grp <= KM_MAXG && nd <= KR_MAXD;
  std::vector<KSJob> sorted_jobs;
  if (by_key) {
    sorted_jobs = jobs;
    std::stable_sort(sorted_jobs.begin(), sorted_jobs.end(), [](const KSJob& x, const KSJob& y) {
      return x.key != y.key ? x.key < y.key : x.g < y.g;
    });
  }
  const std::vector<KSJob>& jl = by_key ? sorted_jobs : jobs;
  ProfScope ps(c, "ks_masked");
  // one accumulator on the key basis per output, summed over every chunk
  uint64_t* A = (uint64_t*)dev_scratch(c, S_KM_A, (size_t)n_grp * 2 * ext * N * 8);
  zero_fill(c, A, (size_t)n_grp * 2 * ext * N);
  const size_t per_job = 0;   // a job's products go straight into its output's accumulator
  const size_t per_src = (size_t)(nd * ext + l1) * N * 8;
  DigitTables dt{};
  for (int d = 0; d < nd; ++d) {
    const BConv& bc = get_modup(c, level, d);
    dt.tab[d] = bc.dev;
    dt.idx[d] = bc.idx;
    dt.n_src[d] = bc.n_src;
    dt.n_dst[d] = bc.n_dst;
  }
  size_t a = 0;
  while (a < jl.size()) {
    std::vector<int> local(sources.size(), -1);
    std::vector<const uint64_t*> srcs;
    std::vector<KSJob> cj;
    size_t b = a, bytes = 0;
    while (b < jl.size()) {
      const bool new_src = local[jl[b].src] < 0;
      const size_t add = per_job + (new_src ? per_src : 0);
      // a chunk ends between runs of one key when the jobs go key by key
      const bool run_start = !by_key || b == a || jl[b].key != jl[b - 1].key || jl[b].g != jl[b - 1].g;
      if (b > a && run_start && bytes + add > KS_BUDGET) break;
      bytes += add;
      if (new_src) {
        local[jl[b].src] = (int)srcs.size();
        srcs.push_back(sources[jl[b].src]);
      }
      KSJob jc = jl[b];
      jc.src = local[jc.src];
      cj.push_back(jc);
      ++b;
    }
    // this chunk's job ranges per output, each pointing at the output's accumulator
    std::vector<GroupDesc> gds;
    if (by_key) {
      for (int g = 0; g < n_grp; ++g) gds.push_back(GroupDesc{A + (size_t)g * 2 * ext * N, 0, 0, 1, 0});
    } else {
      for (size_t r = 0; r < cj.size(); ++r) {
        const int g = cj[r].grp;
        if (r == 0 || cj[r - 1].grp != g)
          gds.push_back(GroupDesc{A + (size_t)g * 2 * ext * N, (int)r, (int)r + 1, 1, 0});
        else
          gds.back().end = (int)r + 1;
      }
    }
    const int U = (int)srcs.size();
    KSJob* jd = upload(c, S_KB_JOBS, cj);
    const uint64_t* const* sd = upload(c, S_KB_SRC, srcs);
    GroupDesc* gd = upload(c, S_KM_CGRP, gds);
    uint64_t* tmp = (uint64_t*)dev_scratch(c, S_KB_TMP, (size_t)U * l1 * N * 8);
    uint64_t* D = (uint64_t*)dev_scratch(c, S_KB_D, (size_t)U * nd * ext * N * 8);
    {
      ProfScope pm(c, "modup");
      hipLaunchKernelGGL(k_gather, dim3(N / KB, l1, U), dim3(KB), 0, c->stream, tmp, sd, l1, c->log_n);
      HIPCHECK(hipGetLastError());
      ntt_inv(c, tmp, l1, lm_q(l1), U, (size_t)l1 * N);
      hipLaunchKernelGGL(k_modup_conv, dim3(N / KB, nd, U), dim3(KB), 0, c->stream, tmp, sd, D, dt, c->alpha, l1, ext,
                         nd, c->L, c->log_n, c->t.mods);
      HIPCHECK(hipGetLastError());
      ntt_fwd(c, D, ext, lm_ext(level, c->L), U * nd, (size_t)ext * N, c->alpha, l1);
    }
    {
      ProfScope pk(c, "keymac");
      if (gds.size() > 65535) FICGCN_THROW(EINVAL_, "too many outputs in one launch");
      const int n_jb = (int)(N / KB), ng = (int)gds.size();
      if (by_key) {
        // each key read once for every output that uses it; runs split in segments for parallelism
        const std::vector<int> runs = key_runs(cj);
        const int n_runs = (int)runs.size() - 1;
        const int n_seg = std::max(1, std::min(32, n_runs / 8));
        std::vector<int> kgl(cj.size());
        for (size_t r = 0; r < cj.size(); ++r) kgl[r] = cj[r].grp;
        const int* rd = upload(c, S_KM_RUNS, runs);
        const int* gld_ = upload(c, S_KM_GL, kgl);
        uint64_t* P = (uint64_t*)dev_scratch(c, S_KM_P, (size_t)n_seg * ng * 2 * ext * N * 8);
        const dim3 grid(n_jb, ext, n_seg);
        int fq = 1;   // the Q limbs in fp64 residues when every Q prime of the level lies in (2^49, 2^50)
        for (int qi = 0; qi < l1; ++qi) fq = fq && c->mod[qi] > (1ull << 49) && c->mod[qi] < (1ull << 50);
#define KM_LAUNCH(NDV, NGV)                                                                                \
  hipLaunchKernelGGL((k_keymac_masked_runs<NDV, NGV>), grid, dim3(KB), 0, c->stream, D, jd, rd, n_runs, n_seg, gld_, \
                     ng, P, ext, l1, c->L, c->n_mod(), c->log_n, fq, c->t.mods)
#define KM_BY_G(NDV)             \
  switch (ng) {                  \
    case 1: KM_LAUNCH(NDV, 1); break; \
    case 2: KM_LAUNCH(NDV, 2); break; \
    case 3: KM_LAUNCH(NDV, 3); break; \
    default: KM_LAUNCH(NDV, 4);  \
  }
        switch (nd) {
          case 1: KM_BY_G(1); break;
          case 2: KM_BY_G(2); break;
          case 3: KM_BY_G(3); break;
          case 4: KM_BY_G(4); break;
          case 5: KM_BY_G(5); break;
          case 6: KM_BY_G(6); break;
          case 7: KM_BY_G(7); break;
          default: KM_BY_G(8);
        }
#undef KM_BY_G
#undef KM_LAUNCH
        HIPCHECK(hipGetLastError());
        hipLaunchKernelGGL(k_masked_combine, dim3(n_jb, ext, 2 * ng), dim3(KB), 0, c->stream, gd, P, ng, n_seg, ext,
                           l1, c->L, c->log_n, c->t.mods);
      } else {
        const bool xcd = n_jb % 8 == 0 && (size_t)n_jb * ng < ((size_t)1 << 31);
        const dim3 grid = xcd ? dim3(n_jb * ng, ext, 1) : dim3(n_jb, ext, ng);
        hipLaunchKernelGGL(k_keymac_masked, grid, dim3(KB), 0, c->stream, D, jd, gd, nd, ext, l1, c->L, c->n_mod(),
                           c->log_n, ng, xcd ? 1 : 0, c->t.mods);
      }
      HIPCHECK(hipGetLastError());
    }
    stream_sync(c);
    a = b;
  }
  // one ModDown per output: P limbs to coefficient form, rounded conversion,
  // forward NTT, then out (+)= (A_Q - conv) P^-1 + sum sigma(add0) (.) pt
  {
    ProfScope pd(c, "moddown");
    const MDK k = mdk(c, level);
    const BConv& md = get_moddown(c, level);
    std::vector<MaskGroup> mg(n_grp, MaskGroup{0, 0});
    for (size_t r = 0; r < jobs.size(); ++r) {
      const int g = jobs[r].grp;
      if (mg[g].end == 0) mg[g].start = (int)r;
      mg[g].end = (int)r + 1;
    }
    KSJob* jall = upload(c, S_KM_JOBS, jobs);
    MaskGroup* mgd = upload(c, S_KM_GRP, mg);
    uint64_t* const* od = upload(c, S_KM_OUT, outs);
    uint64_t* conv = (uint64_t*)dev_scratch(c, S_KM_CONV, (size_t)n_grp * 2 * l1 * N * 8);
    ntt_inv(c, A + (size_t)l1 * N, c->alpha, LimbMap{c->L, 1 << 30, 0}, 2 * n_grp, (size_t)ext * N);
    hipLaunchKernelGGL(k_moddown_conv_batch, dim3(N / KB, 2 * n_grp), dim3(KB), 0, c->stream, A, ext, l1, md.idx,
                       md.idx + md.n_src, md.n_src, (const uint64_t*)md.dev, k, conv, c->log_n, c->t.mods);
    HIPCHECK(hipGetLastError());
    ntt_fwd(c, conv, l1, lm_q(l1), 2 * n_grp, (size_t)l1 * N);
    hipLaunchKernelGGL(k_masked_final, dim3(N / KB, l1, 2 * n_grp), dim3(KB), 0, c->stream, A, conv, ext, l1, k, jall,
                       mgd, od, accumulate ? 1 : 0, c->log_n, c->t.mods);
    HIPCHECK(hipGetLastError());
    stream_sync(c);
  }
}

// ---- batched ciphertext kernels --------------------------------------------------

// d = (x0 y0, x0 y1 + x1 y0, x1 y1) per job, [3][l1][N]
__global__ void k_tensor_batch(const TensorJob* __restrict__ jobs, int l1, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int i = blockIdx.y;
  const TensorJob jb = jobs[blockIdx.z];
  const Mod m = mods[i];
  const size_t o0 = i * N + j, o1 = (l1 + i) * N + j;
  const uint64_t x0 = gld(jb.x + o0), x1 = gld(jb.x + o1), y0 = gld(jb.y + o0), y1 = gld(jb.y + o1);
  gst(jb.d + o0, reduce128((u128)x0 * y0, m));
  gst(jb.d + o1, reduce128((u128)x0 * y1 + (u128)x1 * y0, m));
  gst(jb.d + (2 * l1 + i) * N + j, reduce128((u128)x1 * y1, m));
}

void tensor_batch(ckks_ctx* c, int level, const std::vector<TensorJob>& jobs) {
  if (jobs.empty()) return;
  TensorJob* jd = upload(c, S_TB_JOBS, jobs);
  hipLaunchKernelGGL(k_tensor_batch, dim3(c->N / KB, level + 1, jobs.size()), dim3(KB), 0, c->stream, jd, level + 1,
                     c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
  stream_sync(c);
}

struct RSK {
  uint64_t h[64];               // floor(q_l / 2) mod q_i
  uint64_t inv[64], inv_s[64];  // q_l^-1 mod q_i, Shoup
};

__global__ void k_rs_gather(uint64_t* __restrict__ last, uint64_t* const* __restrict__ cts, int lvl, int log_n) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int z = blockIdx.y;   // ct * 2 + component
  last[(size_t)z * N + j] = gld(cts[z >> 1] + ((size_t)(z & 1) * (lvl + 1) + lvl) * N + j);
}

// d[z][i] = (h - ((x + h) mod q_l)) mod q_i for the last limb x in coefficient form
__global__ void k_rs_prep(const uint64_t* __restrict__ last, uint64_t* __restrict__ d, int lvl, uint64_t hl, RSK k,
                          int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int i = blockIdx.y, z = blockIdx.z;
  const uint64_t ql = mods[lvl].q, q = mods[i].q;
  const uint64_t y = add_mod(last[(size_t)z * N + j], hl, ql);   // < q_l < q_i (descending chain)
  d[((size_t)z * lvl + i) * N + j] = sub_mod(k.h[i], y, q);
}

// c'_i = (c_i + d_i) q_l^-1, compacted in place from [2][l+1][N] to [2][l][N].
// One thread walks the limbs of one component upwards, so a limb is read
// before the write of the next-lower position reaches it; the two
// components write disjoint ranges.
__global__ void k_rs_final(uint64_t* const* __restrict__ cts, const uint64_t* __restrict__ d, int lvl, RSK k, int log_n,
                           const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int z = blockIdx.y;
  const int comp = z & 1;
  uint64_t* ct = cts[z >> 1];
  for (int i = 0; i < lvl; ++i) {
    const uint64_t q = mods[i].q;
    const uint64_t v = add_mod(gld(ct + ((size_t)comp * (lvl + 1) + i) * N + j), d[((size_t)z * lvl + i) * N + j], q);
    gst(ct + ((size_t)comp * lvl + i) * N + j, mul_shoup(v, k.inv[i], k.inv_s[i], q));
  }
}

void rescale_batch(ckks_ctx* c, int level, const std::vector<uint64_t*>& cts) {
  if (cts.empty()) return;
  if (level < 1) FICGCN_THROW(ELEVEL_, "rescale at level 0");
  if (level > 63) FICGCN_THROW(EINVAL_, "too many primes");
  ProfScope ps(c, "rescale");
  const size_t N = c->N;
  const int n = (int)cts.size();
  uint64_t* const* cd = upload(c, S_RS_PTR, cts);
  uint64_t* last = (uint64_t*)dev_scratch(c, S_RS_LAST, (size_t)2 * n * N * 8);
  uint64_t* d = (uint64_t*)dev_scratch(c, S_RS_D, (size_t)2 * n * level * N * 8);
  hipLaunchKernelGGL(k_rs_gather, dim3(N / KB, 2 * n), dim3(KB), 0, c->stream, last, cd, level, c->log_n);
  HIPCHECK(hipGetLastError());
  ntt_inv(c, last, 1, LimbMap{level, 1 << 30, 0}, 2 * n, N);
  RSK k{};
  const uint64_t ql = c->mod[level], hl = ql / 2;
  for (int i = 0; i < level; ++i) {
    const uint64_t q = c->mod[i];
    k.h[i] = hl % q;
    k.inv[i] = invmod(ql % q, q);
    k.inv_s[i] = shoup(k.inv[i], q);
  }
  hipLaunchKernelGGL(k_rs_prep, dim3(N / KB, level, 2 * n), dim3(KB), 0, c->stream, last, d, level, hl, k, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
  ntt_fwd(c, d, level, lm_q(level), 2 * n, (size_t)level * N);
  hipLaunchKernelGGL(k_rs_final, dim3(N / KB, 2 * n), dim3(KB), 0, c->stream, cd, d, level, k, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
  stream_sync(c);
}

// Two rescales in one call, c'' = round(round(c / q_l) / q_{l-1}), word for
// word.  With x_l and x_{l-1} the last two limbs in coefficient form,
//   d_i = (h_l - [x_l + h_l]_{q_l}) mod q_i            (first correction),
//   y   = (x_{l-1} + d_{l-1}) q_l^-1 mod q_{l-1}        (limb l-1 after it),
//   e_i = (h_{l-1} - [y + h_{l-1}]_{q_{l-1}}) mod q_i   (second correction),
// and, the NTT being linear modulo each q_i, for i < l - 1
//   c''_i = c_i (q_l q_{l-1})^-1 + NTT_i((d_i q_l^-1 + e_i) q_{l-1}^-1)  mod q_i,
// which is what two rescales in a row compute, with one forward NTT of l - 1
// limbs instead of l + (l - 1).  h_k = floor(q_k / 2).
constexpr int RS2_MAX = 32;
struct RSK2 {
  uint64_t h1[RS2_MAX], h2[RS2_MAX];            // h_l, h_{l-1} mod q_i
  uint64_t inv1[RS2_MAX], inv1_s[RS2_MAX];      // q_l^-1 mod q_i, Shoup
  uint64_t inv2[RS2_MAX], inv2_s[RS2_MAX];      // q_{l-1}^-1 mod q_i
  uint64_t inv12[RS2_MAX], inv12_s[RS2_MAX];    // (q_l q_{l-1})^-1 mod q_i
};

// last[z][0] = limb l-1, last[z][1] = limb l of component z
__global__ void k_rs2_gather(uint64_t* __restrict__ last, uint64_t* const* __restrict__ cts, int lvl, int log_n) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int z = blockIdx.y, u = blockIdx.z;   // z = ct * 2 + component; u = 0: limb l-1, 1: limb l
  last[((size_t)z * 2 + u) * N + j] = gld(cts[z >> 1] + ((size_t)(z & 1) * (lvl + 1) + lvl - 1 + u) * N + j);
}

// f[z][i] = (d_i q_l^-1 + e_i) q_{l-1}^-1 mod q_i for i < l - 1, coefficient form
__global__ void k_rs2_prep(const uint64_t* __restrict__ last, uint64_t* __restrict__ f, int lvl, RSK2 k, int log_n,
                           const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int i = blockIdx.y, z = blockIdx.z;
  const uint64_t ql = mods[lvl].q, qm = mods[lvl - 1].q, q = mods[i].q;
  const uint64_t xm = last[((size_t)z * 2 + 0) * N + j], xl = last[((size_t)z * 2 + 1) * N + j];
  const uint64_t y1 = add_mod(xl, ql / 2, ql);                        // < q_l < q_{l-1} < q_i (descending chain)
  const uint64_t dm = sub_mod(k.h1[lvl - 1], y1, qm);
  const uint64_t y = mul_shoup(add_mod(xm, dm, qm), k.inv1[lvl - 1], k.inv1_s[lvl - 1], qm);
  const uint64_t y2 = add_mod(y, qm / 2, qm);                         // < q_{l-1} < q_i
  const uint64_t d = sub_mod(k.h1[i], y1, q), e = sub_mod(k.h2[i], y2, q);
  const uint64_t t = add_mod(mul_shoup(d, k.inv1[i], k.inv1_s[i], q), e, q);
  f[((size_t)z * (lvl - 1) + i) * N + j] = mul_shoup(t, k.inv2[i], k.inv2_s[i], q);
}

// c''_i = c_i (q_l q_{l-1})^-1 + f_i, compacted in place from [2][l+1][N] to
// [2][l-1][N]: one thread walks the limbs of one component upwards, so each
// write lands on a limb this thread has already read (or on a dropped limb of
// the first component, which no thread reads).
__global__ void k_rs2_final(uint64_t* const* __restrict__ cts, const uint64_t* __restrict__ f, int lvl, RSK2 k,
                            int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)KB + threadIdx.x;
  const int z = blockIdx.y;
  const int comp = z & 1;
  uint64_t* ct = cts[z >> 1];
  for (int i = 0; i < lvl - 1; ++i) {
    const uint64_t q = mods[i].q;
    const uint64_t v = mul_shoup(gld(ct + ((size_t)comp * (lvl + 1) + i) * N + j), k.inv12[i], k.inv12_s[i], q);
    gst(ct + ((size_t)comp * (lvl - 1) + i) * N + j, add_mod(v, f[((size_t)z * (lvl - 1) + i) * N + j], q));
  }
}

void rescale2_batch(ckks_ctx* c, int level, const std::vector<uint64_t*>& cts) {
  if (cts.empty()) return;
  if (level < 2 || level > RS2_MAX) {
    rescale_batch(c, level, cts);
    rescale_batch(c, level - 1, cts);
    return;
  }
  ProfScope ps(c, "rescale");
  const size_t N = c->N;
  const int n = (int)cts.size();
  uint64_t* const* cd = upload(c, S_RS_PTR, cts);
  uint64_t* last = (uint64_t*)dev_scratch(c, S_RS_LAST, (size_t)2 * n * 2 * N * 8);
  uint64_t* f = (uint64_t*)dev_scratch(c, S_RS_D, (size_t)2 * n * (level - 1) * N * 8);
  hipLaunchKernelGGL(k_rs2_gather, dim3(N / KB, 2 * n, 2), dim3(KB), 0, c->stream, last, cd, level, c->log_n);
  HIPCHECK(hipGetLastError());
  ntt_inv(c, last, 2, LimbMap{level - 1, 1 << 30, 0}, 2 * n, 2 * N);
  RSK2 k{};
  const uint64_t ql = c->mod[level], qm = c->mod[level - 1];
  for (int i = 0; i < level; ++i) {
    const uint64_t q = c->mod[i];
    k.h1[i] = (ql / 2) % q;
    k.inv1[i] = invmod(ql % q, q);
    k.inv1_s[i] = shoup(k.inv1[i], q);
    if (i < level - 1) {
      k.h2[i] = (qm / 2) % q;
      k.inv2[i] = invmod(qm % q, q);
      k.inv2_s[i] = shoup(k.inv2[i], q);
      k.inv12[i] = (uint64_t)((u128)k.inv1[i] * k.inv2[i] % q);
      k.inv12_s[i] = shoup(k.inv12[i], q);
    }
  }
  hipLaunchKernelGGL(k_rs2_prep, dim3(N / KB, level - 1, 2 * n), dim3(KB), 0, c->stream, last, f, level, k, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
  ntt_fwd(c, f, level - 1, lm_q(level - 1), 2 * n, (size_t)(level - 1) * N);
  hipLaunchKernelGGL(k_rs2_final, dim3(N / KB, 2 * n), dim3(KB), 0, c->stream, cd, f, level, k, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
  stream_sync(c);
}

// outs[g] (+)= sum over the terms of group g of ct (.) pt, or ct when pt is null
__global__ void k_group_mac(const MacTerm* __restrict__ terms, const int* __restrict__ group_start,
                            uint64_t* const* __restrict__ outs, int l1, int accumulate, int log_n, int n_groups,
                            int xcd_order, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  // limb slowest: one limb of every group's terms is in flight at a time.
  // With xcd_order, blocks go round-robin over the 8 XCDs by linear id, so
  // block b runs coefficient block 8 (b / 8 / n_groups) + b % 8 for group
  // (b / 8) % n_groups: every group of one coefficient block runs on one XCD,
  // back to back, and the ciphertexts the groups share (baby steps) are read
  // into that XCD's L2 once.  One thread takes both components of a
  // coefficient: each plaintext word is read once for the two products.
  const int i = blockIdx.z;
  int jb, g;
  if (xcd_order) {
    const int b = blockIdx.x, idx = b >> 3;
    jb = (b & 7) + 8 * (idx / n_groups);
    g = idx % n_groups;
  } else {
    jb = blockIdx.x;
    g = blockIdx.y;
  }
  const size_t j = (size_t)jb * KB + threadIdx.x;
  const Mod m = mods[i];
  const size_t o0 = (size_t)i * N + j, o1 = ((size_t)l1 + i) * N + j;
  uint64_t* out = outs[g];
  uint64_t a0 = accumulate ? gld(out + o0) : 0, a1 = accumulate ? gld(out + o1) : 0;
  // A term without a plaintext adds its ciphertext: it is multiplied by a
  // stored 1 instead (the words are below q, so the sum is the same), which
  // keeps the term loop free of branches.  Terms go in fours: the twelve loads
  // of four terms are issued before their products, summed in 128 bits and
  // reduced once per four.
  const size_t pj = (size_t)i * N + j;
  auto load = [&](int t, uint64_t& x0, uint64_t& x1, uint64_t& p) {
    const MacTerm tm = terms[t];
    x0 = gld(tm.ct + (tm.l1 ? pj : o0));
    x1 = gld(tm.ct + (tm.l1 ? ((size_t)tm.l1 + i) * N + j : o1));
    p = gld(tm.pt ? tm.pt + pj : &k_one_word);
  };
  const int t_end = group_start[g + 1];
  int t = group_start[g];
  for (; t + 4 <= t_end; t += 4) {
    uint64_t x0[4], x1[4], p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) load(t + u, x0[u], x1[u], p[u]);
    u128 s0 = 0, s1 = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0 += (u128)x0[u] * p[u];
      s1 += (u128)x1[u] * p[u];
    }
    a0 = add_mod(a0, reduce128(s0, m), m.q);
    a1 = add_mod(a1, reduce128(s1, m), m.q);
  }
  u128 s0 = 0, s1 = 0;
  for (; t < t_end; ++t) {
    uint64_t x0, x1, p;
    load(t, x0, x1, p);
    s0 += (u128)x0 * p;
    s1 += (u128)x1 * p;
  }
  gst(out + o0, add_mod(a0, reduce128(s0, m), m.q));
  gst(out + o1, add_mod(a1, reduce128(s1, m), m.q));
}

void group_mac(ckks_ctx* c, int level, const std::vector<std::vector<MacTerm>>& groups,
               const std::vector<uint64_t*>& outs, bool accumulate) {
  if (groups.empty()) return;
  if (groups.size() != outs.size()) FICGCN_THROW(EINVAL_, "group/output count mismatch");
  ProfScope ps(c, "group_mac");
  std::vector<MacTerm> flat;
  std::vector<int> start{0};
  for (const auto& g : groups) {
    for (const MacTerm& t : g)
      if (!t.ct) FICGCN_THROW(EINVAL_, "null term");
    flat.insert(flat.end(), g.begin(), g.end());
    start.push_back((int)flat.size());
  }
  for (uint64_t* o : outs)
    if (!o) FICGCN_THROW(EINVAL_, "null output");
  MacTerm* td = upload(c, S_GM_TERMS, flat);
  int* sd = upload(c, S_GM_START, start);
  uint64_t* const* od = upload(c, S_GM_OUT, outs);
  if (groups.size() > 65535) FICGCN_THROW(EINVAL_, "too many groups in one launch");
  const int n_jb = c->N / KB, ng = (int)groups.size();
  const bool xcd = n_jb % 8 == 0 && (size_t)n_jb * ng < ((size_t)1 << 31);
  const dim3 grid = xcd ? dim3(n_jb * ng, 1, level + 1) : dim3(n_jb, ng, level + 1);
  hipLaunchKernelGGL(k_group_mac, grid, dim3(KB), 0, c->stream, td, sd, od, level + 1, accumulate ? 1 : 0, c->log_n, ng,
                     xcd ? 1 : 0, c->t.mods);
  HIPCHECK(hipGetLastError());
  stream_sync(c);
}


// ---- masked sums of several ciphertexts under shared masks ----------------------

// outs[g * NP + c] (+)= sum over the terms of group g of ct_c (.) pt (ct_c alone when pt is
// null).  The NP ciphertexts of a term share its plaintext word, read once; a thread takes
// two neighbouring coefficients of one limb with 16-byte loads, so every load instruction
// moves two words and NP + 1 streams are in flight per term.
// GM_TB threads per block: the baby-step ciphertexts of one block's 2 GM_TB coefficients
// (every packed ciphertext, both components) stay in L2 while the masks stream past them.
//
// Products, by the level's primes: all in (2^49, 2^50) (AR = 2): fp64 residues, each
// product an exact signed representative in (-q, q) from one fp64 product and its fma
// error term (fpmod.h), summed in doubles and brought back every six terms; the 24
// accumulators take a third of the registers of the integer forms, so five waves fit
// per SIMD instead of three.  All below 2^50 (AR = 1): a word w < 2^50 is split into
// w0 = w mod 2^25 and w1 = floor(w / 2^25), both below 2^25, and
//   x p = x0 p0 + (x0 p1 + x1 p0) 2^25 + x1 p1 2^50;
// the three partial sums are kept in 64-bit registers, each partial product added by one
// 32 x 32 + 64 multiply-add (every partial below 2^51, so GM_MAX_TERMS terms fit), and the
// group's sum is assembled to 128 bits and reduced once at the end.  Otherwise (AR = 0,
// wider primes) products are summed in 128 bits and reduced every four terms.
constexpr int GM_TB = 128;
constexpr int GM_MAX_TERMS = 8191;   // 64-bit partial sums: 8191 * 2^51 < 2^64

template <int NP, int AR>
__global__ void __launch_bounds__(GM_TB) k_group_mac_np(const MacTermNP* __restrict__ terms, const int* __restrict__ group_start,
                               uint64_t* const* __restrict__ outs, int l1, int accumulate, int log_n, int n_groups,
                               int xcd_order, const Mod* __restrict__ mods) {
  typedef uint64_t v2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(1))) const v2 gv2;
  typedef __attribute__((address_space(1))) v2 gv2w;
  const size_t N = (size_t)1 << log_n;
  const int i = blockIdx.z;
  int jb, g;
  if (xcd_order) {   // every group of one coefficient block back to back on one XCD
    const int b = blockIdx.x, idx = b >> 3;
    jb = (b & 7) + 8 * (idx / n_groups);
    g = idx % n_groups;
  } else {
    jb = blockIdx.x;
    g = blockIdx.y;
  }
  const size_t j = 2 * ((size_t)jb * GM_TB + threadIdx.x);
  const Mod m = mods[i];
  const size_t o0 = (size_t)i * N + j, o1 = ((size_t)l1 + i) * N + j;
  const int t_end = group_start[g + 1];
  int t = group_start[g];
  // per ciphertext, the four words of a thread: component 0 at j, j+1, component 1 at j, j+1
  uint64_t res[NP][4];
  if (AR == 2) {
    // fp64 residues (every prime in (2^49, 2^50)): each product a signed representative in
    // (-q, q), summed in a double; six terms at most between reductions keep every sum an
    // exact integer below 2^53
    const double qd = (double)m.q, qinv = 1.0 / qd;
    double S[NP][4];
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) S[c][k] = 0.0;
    auto cv = [](uint64_t v) { return b2f(to_fbits(v)); };
    auto mac = [&](const v2& p, const v2 (&x)[NP], const v2 (&y)[NP]) {
      const double p0 = cv(p.x), p1 = cv(p.y);
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        S[c][0] += fmulmod_s(cv(x[c].x), p0, qd, qinv);
        S[c][1] += fmulmod_s(cv(x[c].y), p1, qd, qinv);
        S[c][2] += fmulmod_s(cv(y[c].x), p0, qd, qinv);
        S[c][3] += fmulmod_s(cv(y[c].y), p1, qd, qinv);
      }
    };
    auto fold = [&]() {
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) S[c][k] = sred(S[c][k], qd, qinv);
    };
    int cnt = 0;
    for (; t + 2 <= t_end; t += 2) {
      const MacTermNP ta = terms[t], tb = terms[t + 1];
      v2 pa = {1, 1}, pb = {1, 1};
      if (ta.pt) pa = __builtin_nontemporal_load((gv2*)(ta.pt + (size_t)i * N + j));
      if (tb.pt) pb = __builtin_nontemporal_load((gv2*)(tb.pt + (size_t)i * N + j));
      v2 xa[NP], ya[NP], xb[NP], yb[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        xa[c] = *(gv2*)(ta.ct[c] + o0);
        ya[c] = *(gv2*)(ta.ct[c] + o1);
        xb[c] = *(gv2*)(tb.ct[c] + o0);
        yb[c] = *(gv2*)(tb.ct[c] + o1);
      }
      mac(pa, xa, ya);
      mac(pb, xb, yb);
      if ((cnt += 2) == 6) {
        fold();
        cnt = 0;
      }
    }
    if (t < t_end) {
      const MacTermNP ta = terms[t];
      v2 pa = {1, 1};
      if (ta.pt) pa = __builtin_nontemporal_load((gv2*)(ta.pt + (size_t)i * N + j));
      v2 xa[NP], ya[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        xa[c] = *(gv2*)(ta.ct[c] + o0);
        ya[c] = *(gv2*)(ta.ct[c] + o1);
      }
      mac(pa, xa, ya);
    }
    fold();
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) res[c][k] = from_fbits(f2b(canon(S[c][k], qd)));
  } else if (AR == 1) {
    constexpr uint32_t M25 = (1u << 25) - 1;
    uint64_t A[NP][4], B[NP][4], C[NP][4];
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) A[c][k] = B[c][k] = C[c][k] = 0;
    auto part = [&](uint64_t& a, uint64_t& b, uint64_t& cc, uint64_t w, uint32_t p0, uint32_t p1) {
      const uint32_t w0 = (uint32_t)w & M25, w1 = (uint32_t)(w >> 25);
      a += (uint64_t)w0 * p0;
      b += (uint64_t)w0 * p1;
      b += (uint64_t)w1 * p0;
      cc += (uint64_t)w1 * p1;
    };
    auto mac = [&](const v2& p, const v2 (&x)[NP], const v2 (&y)[NP]) {
      const uint32_t px0 = (uint32_t)p.x & M25, px1 = (uint32_t)(p.x >> 25);
      const uint32_t py0 = (uint32_t)p.y & M25, py1 = (uint32_t)(p.y >> 25);
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        part(A[c][0], B[c][0], C[c][0], x[c].x, px0, px1);
        part(A[c][1], B[c][1], C[c][1], x[c].y, py0, py1);
        part(A[c][2], B[c][2], C[c][2], y[c].x, px0, px1);
        part(A[c][3], B[c][3], C[c][3], y[c].y, py0, py1);
      }
    };
    for (; t + 2 <= t_end; t += 2) {
      const MacTermNP ta = terms[t], tb = terms[t + 1];
      v2 pa = {1, 1}, pb = {1, 1};
      // each mask word is read once: streamed past the cache so that the baby-step words,
      // which every giant step of this coefficient block reads again, stay in L2
      if (ta.pt) pa = __builtin_nontemporal_load((gv2*)(ta.pt + (size_t)i * N + j));
      if (tb.pt) pb = __builtin_nontemporal_load((gv2*)(tb.pt + (size_t)i * N + j));
      v2 xa[NP], ya[NP], xb[NP], yb[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        xa[c] = *(gv2*)(ta.ct[c] + o0);
        ya[c] = *(gv2*)(ta.ct[c] + o1);
        xb[c] = *(gv2*)(tb.ct[c] + o0);
        yb[c] = *(gv2*)(tb.ct[c] + o1);
      }
      mac(pa, xa, ya);
      mac(pb, xb, yb);
    }
    if (t < t_end) {
      const MacTermNP ta = terms[t];
      v2 pa = {1, 1};
      if (ta.pt) pa = __builtin_nontemporal_load((gv2*)(ta.pt + (size_t)i * N + j));
      v2 xa[NP], ya[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        xa[c] = *(gv2*)(ta.ct[c] + o0);
        ya[c] = *(gv2*)(ta.ct[c] + o1);
      }
      mac(pa, xa, ya);
    }
#pragma unroll
    for (int c = 0; c < NP; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        res[c][k] = reduce128((u128)A[c][k] + ((u128)B[c][k] << 25) + ((u128)C[c][k] << 50), m);
  } else {
    u128 s[NP][4];
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      res[c][0] = res[c][1] = res[c][2] = res[c][3] = 0;
      s[c][0] = s[c][1] = s[c][2] = s[c][3] = 0;
    }
    auto mac = [&](const v2& p, const v2 (&x)[NP], const v2 (&y)[NP]) {
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        s[c][0] += (u128)x[c].x * p.x;
        s[c][1] += (u128)x[c].y * p.y;
        s[c][2] += (u128)y[c].x * p.x;
        s[c][3] += (u128)y[c].y * p.y;
      }
    };
    auto fold = [&]() {
#pragma unroll
      for (int c = 0; c < NP; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          res[c][k] = add_mod(res[c][k], reduce128(s[c][k], m), m.q);
          s[c][k] = 0;
        }
    };
    // two terms' loads in flight together; products of four terms summed in 128 bits
    // (each below 2^124 for words below 2^62) before one reduction
    int cnt = 0;
    for (; t + 2 <= t_end; t += 2) {
      const MacTermNP ta = terms[t], tb = terms[t + 1];
      v2 pa = {1, 1}, pb = {1, 1};
      if (ta.pt) pa = *(gv2*)(ta.pt + (size_t)i * N + j);
      if (tb.pt) pb = *(gv2*)(tb.pt + (size_t)i * N + j);
      v2 xa[NP], ya[NP], xb[NP], yb[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        xa[c] = *(gv2*)(ta.ct[c] + o0);
        ya[c] = *(gv2*)(ta.ct[c] + o1);
        xb[c] = *(gv2*)(tb.ct[c] + o0);
        yb[c] = *(gv2*)(tb.ct[c] + o1);
      }
      mac(pa, xa, ya);
      mac(pb, xb, yb);
      if ((cnt += 2) == 4) {
        fold();
        cnt = 0;
      }
    }
    if (t < t_end) {
      const MacTermNP ta = terms[t];
      v2 pa = {1, 1};
      if (ta.pt) pa = *(gv2*)(ta.pt + (size_t)i * N + j);
      v2 xa[NP], ya[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) {
        xa[c] = *(gv2*)(ta.ct[c] + o0);
        ya[c] = *(gv2*)(ta.ct[c] + o1);
      }
      mac(pa, xa, ya);
    }
    fold();
  }
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    uint64_t* out = outs[(size_t)g * NP + c];
    if (accumulate) {
      const v2 u = *(gv2*)(out + o0), v = *(gv2*)(out + o1);
      res[c][0] = add_mod(res[c][0], u.x, m.q);
      res[c][1] = add_mod(res[c][1], u.y, m.q);
      res[c][2] = add_mod(res[c][2], v.x, m.q);
      res[c][3] = add_mod(res[c][3], v.y, m.q);
    }
    const v2 r0 = {res[c][0], res[c][1]}, r1 = {res[c][2], res[c][3]};
    *(gv2w*)(out + o0) = r0;
    *(gv2w*)(out + o1) = r1;
  }
}

void group_mac_np(ckks_ctx* c, int level, int np, const std::vector<std::vector<MacTermNP>>& groups,
                  const std::vector<uint64_t*>& outs, bool accumulate) {
  if (groups.empty()) return;
  if (np < 1 || np > MacTermNP::MAX) FICGCN_THROW(EINVAL_, "shared-mask sum: 1 to 4 ciphertexts per term");
  if (outs.size() != groups.size() * np) FICGCN_THROW(EINVAL_, "group/output count mismatch");
  if (c->N < 2 * GM_TB) FICGCN_THROW(EINVAL_, "ring too small for the shared-mask sum");
  std::vector<MacTermNP> flat;
  std::vector<int> start{0};
  for (const auto& g : groups) {
    for (const MacTermNP& t : g)
      for (int k = 0; k < np; ++k)
        if (!t.ct[k]) FICGCN_THROW(EINVAL_, "null term");
    flat.insert(flat.end(), g.begin(), g.end());
    start.push_back((int)flat.size());
  }
  for (uint64_t* o : outs)
    if (!o) FICGCN_THROW(EINVAL_, "null output");
  MacTermNP* td = upload(c, S_GM_TERMS, flat);
  int* sd = upload(c, S_GM_START, start);
  uint64_t* const* od = upload(c, S_GM_OUT, outs);
  if (groups.size() > 65535) FICGCN_THROW(EINVAL_, "too many groups in one launch");
  const int n_jb = c->N / (2 * GM_TB), ng = (int)groups.size();
  const bool xcd = n_jb % 8 == 0 && (size_t)n_jb * ng < ((size_t)1 << 31);
  const dim3 grid = xcd ? dim3(n_jb * ng, 1, level + 1) : dim3(n_jb, ng, level + 1);
  const int acc = accumulate ? 1 : 0;
  // split-limb products need every prime of the level below 2^50 and at most GM_MAX_TERMS
  // terms per group
  bool l25 = true, f50 = true;
  for (int i = 0; i <= level; ++i) {
    l25 = l25 && c->mod[i] < (1ull << 50);
    f50 = f50 && c->mod[i] > (1ull << 49) && c->mod[i] < (1ull << 50);
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) l25 = l25 && groups[gi].size() <= (size_t)GM_MAX_TERMS;
  const int ar = f50 ? 2 : l25 ? 1 : 0;
  ProfScope ps(c, "bsgs_inner");   // the launch alone (its tables are uploaded above)
#define GM_LAUNCH(NPV, AV)                                                                                     \
  hipLaunchKernelGGL((k_group_mac_np<NPV, AV>), grid, dim3(GM_TB), 0, c->stream, td, sd, od, level + 1, acc, \
                     c->log_n, ng, xcd ? 1 : 0, c->t.mods)
#define GM_BY_AR(NPV)          \
  switch (ar) {                \
    case 0: GM_LAUNCH(NPV, 0); break; \
    case 1: GM_LAUNCH(NPV, 1); break; \
    default: GM_LAUNCH(NPV, 2);       \
  }
  switch (np) {
    case 1: GM_BY_AR(1); break;
    case 2: GM_BY_AR(2); break;
    case 3: GM_BY_AR(3); break;
    default: GM_BY_AR(4);
  }
#undef GM_BY_AR
#undef GM_LAUNCH
  HIPCHECK(hipGetLastError());
  ps.stop();
  stream_sync(c);
}

}  // namespace ficgcn
