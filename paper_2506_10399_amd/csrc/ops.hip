// Elementwise and key-switching kernels (evaluation form unless noted).
//
// Layouts (uint64 words, limb-major, each limb N contiguous words):
//   ciphertext  [2][l+1][N]            over q_0..q_l
//   ModUp D     [beta'][l+1+alpha][N]  digit d extended to Q_l and P
//   key         [beta][2][L+alpha][N]  switching key over every prime
// One thread owns one coefficient index j of one limb, so every access of a
// warp is 64 consecutive words.
#include "internal.h"

namespace ficgcn {

constexpr int EW = 256;

__device__ __forceinline__ uint32_t auto_index(uint32_t k, uint64_t g, int log_n) {
  // evaluation index k holds A(psi^(2 brev(k) + 1)); sigma_g reads the index of psi^(g (2 brev(k) + 1))
  uint32_t N2 = 2u << log_n;
  uint32_t e = 2u * bitrev(k, log_n) + 1u;
  uint32_t ge = (uint32_t)(((uint64_t)e * g) & (N2 - 1));
  return bitrev((ge - 1u) >> 1, log_n);
}

__global__ void k_pmul_acc(uint64_t* __restrict__ acc, PtrList cts, PtrList pts, int k, int n_limbs, int log_n,
                           const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const Mod m = mods[i];
  u128 s = 0;
  for (int t = 0; t < k; ++t) s += (u128)pts.p[t][i * N + j] * cts.p[t][(c * n_limbs + i) * N + j];
  uint64_t* a = acc + (c * n_limbs + i) * N + j;
  *a = add_mod(*a, reduce128(s, m), m.q);
}

void pmul_acc(ckks_ctx* c, uint64_t* acc, const PtrList& cts, const PtrList& pts, int k, int n_limbs) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_pmul_acc, dim3(c->N / EW, n_limbs, 2), dim3(EW), 0, c->stream, acc, cts, pts, k, n_limbs,
                     c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

// consts: [k][n_limbs][2] (residue, Shoup companion)
__global__ void k_smul_acc(uint64_t* __restrict__ acc, PtrList cts, const uint64_t* __restrict__ consts, int k,
                           int n_limbs, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const uint64_t q = mods[i].q;
  uint64_t* a = acc + (c * n_limbs + i) * N + j;
  uint64_t r = *a;
  for (int t = 0; t < k; ++t) {
    const uint64_t* cc = consts + ((size_t)t * n_limbs + i) * 2;
    r = add_mod(r, mul_shoup(cts.p[t][(c * n_limbs + i) * N + j], cc[0], cc[1], q), q);
  }
  *a = r;
}

void smul_acc(ckks_ctx* c, uint64_t* acc, const PtrList& cts, const uint64_t* consts_dev, int k, int n_limbs) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_smul_acc, dim3(c->N / EW, n_limbs, 2), dim3(EW), 0, c->stream, acc, cts, consts_dev, k,
                     n_limbs, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

__global__ void k_add(uint64_t* __restrict__ acc, const uint64_t* __restrict__ in, int n_limbs, int log_n,
                      const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y, p = blockIdx.z;
  const size_t o = (p * n_limbs + i) * N + j;
  acc[o] = add_mod(acc[o], in[o], mods[i].q);
}

void add_inplace(ckks_ctx* c, uint64_t* acc, const uint64_t* in, int n_limbs, int n_polys) {
  hipLaunchKernelGGL(k_add, dim3(c->N / EW, n_limbs, n_polys), dim3(EW), 0, c->stream, acc, in, n_limbs, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
}

__global__ void k_automorph(uint64_t* __restrict__ out, const uint64_t* __restrict__ in, uint64_t g, int n_limbs,
                            int log_n) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * EW + threadIdx.x;
  const size_t base = ((size_t)blockIdx.z * n_limbs + blockIdx.y) * N;
  out[base + j] = in[base + auto_index(j, g, log_n)];
}

void automorph_ntt(ckks_ctx* c, uint64_t* out, const uint64_t* in, uint64_t g, int n_limbs, int n_polys) {
  hipLaunchKernelGGL(k_automorph, dim3(c->N / EW, n_limbs, n_polys), dim3(EW), 0, c->stream, out, in, g, n_limbs,
                     c->log_n);
  HIPCHECK(hipGetLastError());
}

// Fast base conversion in coefficient form.
// table: [ns] hat_inv, [ns] hat_inv_shoup, [nd][ns] hat_mod_dst.
// Destination modulus m is written at limb position (m < L ? m : m - L + lvl1).
__global__ void k_bconv(const uint64_t* __restrict__ src, int ns, size_t src_ps, const int* __restrict__ src_mod,
                        uint64_t* __restrict__ dst, size_t dst_ps, const int* __restrict__ dst_mod, int nd, int lvl1,
                        int L, const uint64_t* __restrict__ table, int log_n, const Mod* __restrict__ mods,
                        int sub_half) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int p = blockIdx.y;
  const uint64_t* s = src + p * src_ps;
  uint64_t y[8];
  for (int t = 0; t < ns; ++t) {
    uint64_t b = mods[src_mod[t]].q;
    y[t] = mul_shoup(s[t * N + j], table[t], table[ns + t], b);
  }
  const uint64_t* hm = table + 2 * ns;
  for (int d = 0; d < nd; ++d) {
    int m = dst_mod[d];
    const Mod md = mods[m];
    u128 acc = 0;
    for (int t = 0; t < ns; ++t) acc += (u128)y[t] * hm[d * ns + t];
    uint64_t r = reduce128(acc, md);
    int pos = m < L ? m : m - L + lvl1;
    dst[p * dst_ps + pos * N + j] = r;
  }
}

struct BConvDev {
  const int* src_mod;
  const int* dst_mod;
};

static BConvDev bconv_indices(ckks_ctx*, const BConv& bc, int) { return BConvDev{bc.idx, bc.idx + bc.n_src}; }

// scratch slots used here (contexts own them)
enum { S_MODUP_TMP = 1, S_IDX_A = 2, S_IDX_B = 3, S_MD_TMP = 4, S_RS_TMP = 5, S_RS_D = 6 };

void modup(ckks_ctx* c, const uint64_t* a_ntt, int level, uint64_t* D, uint64_t* tmp) {
  ProfScope ps(c, "modup");
  const size_t N = c->N;
  const int l1 = level + 1, ext = l1 + c->alpha;
  const int nd = (l1 + c->alpha - 1) / c->alpha;
  if (!tmp) tmp = (uint64_t*)c->buf(S_MODUP_TMP, (size_t)l1 * N * 8);
  HIPCHECK(hipMemcpyAsync(tmp, a_ntt, (size_t)l1 * N * 8, hipMemcpyDeviceToDevice, c->stream));
  ntt_inv(c, tmp, l1, lm_q(l1), 1, 0);
  for (int d = 0; d < nd; ++d) {
    const BConv& bc = get_modup(c, level, d);
    BConvDev idx = bconv_indices(c, bc, S_IDX_A);
    hipLaunchKernelGGL(k_bconv, dim3(N / EW, 1), dim3(EW), 0, c->stream, tmp + (size_t)d * c->alpha * N, bc.n_src,
                       (size_t)0, idx.src_mod, D + (size_t)d * ext * N, (size_t)0, idx.dst_mod, bc.n_dst, l1, c->L,
                       (const uint64_t*)bc.dev, c->log_n, c->t.mods, 0);
    HIPCHECK(hipGetLastError());
    // the digit's own residues are the input limbs (already in evaluation form)
    HIPCHECK(hipMemcpyAsync(D + ((size_t)d * ext + (size_t)d * c->alpha) * N, a_ntt + (size_t)d * c->alpha * N,
                            (size_t)bc.n_src * N * 8, hipMemcpyDeviceToDevice, c->stream));
  }
  ntt_fwd(c, D, ext, lm_ext(level, c->L), nd, (size_t)ext * N, c->alpha, l1);
}

__global__ void k_keymac(uint64_t* __restrict__ acc, const uint64_t* __restrict__ D, const uint64_t* __restrict__ key,
                         int nd, int ext, int lvl1, int L, int n_mod, uint64_t g, int log_n,
                         const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * EW + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const int m = i < lvl1 ? i : i - lvl1 + L;
  const uint32_t jj = g == 1 ? j : auto_index(j, g, log_n);
  u128 s = 0;
  for (int d = 0; d < nd; ++d)
    s += (u128)D[((size_t)d * ext + i) * N + jj] * key[(((size_t)d * 2 + c) * n_mod + m) * N + j];
  acc[((size_t)c * ext + i) * N + j] = reduce128(s, mods[m]);
}

void keymac(ckks_ctx* c, uint64_t* acc, const uint64_t* D, const uint64_t* key, int level, uint64_t g) {
  ProfScope ps(c, "keymac");
  const int l1 = level + 1, ext = l1 + c->alpha;
  const int nd = (l1 + c->alpha - 1) / c->alpha;
  hipLaunchKernelGGL(k_keymac, dim3(c->N / EW, ext, 2), dim3(EW), 0, c->stream, acc, D, key, nd, ext, l1, c->L,
                     c->n_mod(), g, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

struct MDConst {
  uint64_t hP[8];
  uint64_t hQ[64];
  uint64_t pinv[64], pinv_s[64];
};

// conv_c[i] = FastBConv_{P->q_i}([x_P + h]_P) - h  (coefficient form)
__global__ void k_moddown_conv(const uint64_t* __restrict__ accP, size_t acc_ps, const int* __restrict__ src_mod,
                               const int* __restrict__ dst_mod, int ns, int nd, const uint64_t* __restrict__ table,
                               MDConst k, uint64_t* __restrict__ out, size_t out_ps, int log_n,
                               const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int c = blockIdx.y;
  uint64_t y[8];
  for (int t = 0; t < ns; ++t) {
    uint64_t b = mods[src_mod[t]].q;
    uint64_t x = add_mod(accP[c * acc_ps + t * N + j], k.hP[t], b);
    y[t] = mul_shoup(x, table[t], table[ns + t], b);
  }
  const uint64_t* hm = table + 2 * ns;
  for (int d = 0; d < nd; ++d) {
    const Mod md = mods[dst_mod[d]];
    u128 acc = 0;
    for (int t = 0; t < ns; ++t) acc += (u128)y[t] * hm[d * ns + t];
    out[c * out_ps + d * N + j] = sub_mod(reduce128(acc, md), k.hQ[d], md.q);
  }
}

// out_c[i] = (acc_c[i] - conv_c[i]) * P^-1 (+ add_c[i], add0 read through sigma_g when g != 1)
__global__ void k_moddown_final(const uint64_t* __restrict__ acc, size_t acc_ps, const uint64_t* __restrict__ conv,
                                size_t conv_ps, MDConst k, uint64_t* __restrict__ out, size_t out_ps,
                                const uint64_t* __restrict__ add0, uint64_t g0, const uint64_t* __restrict__ add1,
                                int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t j = blockIdx.x * EW + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const uint64_t q = mods[i].q;
  uint64_t v = sub_mod(acc[c * acc_ps + i * N + j], conv[c * conv_ps + i * N + j], q);
  v = mul_shoup(v, k.pinv[i], k.pinv_s[i], q);
  if (c == 0 && add0) v = add_mod(v, add0[i * N + (g0 == 1 ? j : auto_index(j, g0, log_n))], q);
  if (c == 1 && add1) v = add_mod(v, add1[i * N + j], q);
  out[c * out_ps + i * N + j] = v;
}

static MDConst md_const(ckks_ctx* c, int level) {
  MDConst k{};
  if (c->alpha > 8 || level + 1 > 64) FICGCN_THROW(EINVAL_, "too many primes");
  // h = floor(P / 2) = (P - 1) / 2 (P odd); residues via (P mod m - 1) / 2 computed as
  // (P - 1)/2 mod m = (P mod m - 1) * 2^-1 mod m
  for (int t = 0; t < c->alpha; ++t) {
    uint64_t pm = c->mod[c->L + t];
    uint64_t P_mod = 1;
    for (int u = 0; u < c->alpha; ++u) P_mod = (uint64_t)((u128)P_mod * (c->mod[c->L + u] % pm) % pm);
    k.hP[t] = (uint64_t)((u128)sub_mod(P_mod, 1, pm) * invmod(2, pm) % pm);
  }
  for (int i = 0; i <= level; ++i) {
    uint64_t q = c->mod[i];
    uint64_t P_mod = 1;
    for (int u = 0; u < c->alpha; ++u) P_mod = (uint64_t)((u128)P_mod * (c->mod[c->L + u] % q) % q);
    k.hQ[i] = (uint64_t)((u128)sub_mod(P_mod, 1, q) * invmod(2, q) % q);
    k.pinv[i] = invmod(P_mod, q);
    k.pinv_s[i] = shoup(k.pinv[i], q);
  }
  return k;
}

void moddown(ckks_ctx* c, uint64_t* acc, int level, uint64_t* out, const uint64_t* add0, uint64_t g_add0,
             const uint64_t* add1, uint64_t* conv) {
  ProfScope ps(c, "moddown");
  const size_t N = c->N;
  const int l1 = level + 1, ext = l1 + c->alpha;
  // P limbs back to coefficient form
  ntt_inv(c, acc + (size_t)l1 * N, c->alpha, LimbMap{c->L, 1 << 30, 0}, 2, (size_t)ext * N);
  const BConv& bc = get_moddown(c, level);
  BConvDev idx = bconv_indices(c, bc, S_IDX_B);
  MDConst k = md_const(c, level);
  if (!conv) conv = (uint64_t*)c->buf(S_MD_TMP, (size_t)2 * l1 * N * 8);
  hipLaunchKernelGGL(k_moddown_conv, dim3(N / EW, 2), dim3(EW), 0, c->stream, acc + (size_t)l1 * N, (size_t)ext * N,
                     idx.src_mod, idx.dst_mod, bc.n_src, bc.n_dst, (const uint64_t*)bc.dev, k, conv, (size_t)l1 * N,
                     c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
  ntt_fwd(c, conv, l1, lm_q(l1), 2, (size_t)l1 * N);
  hipLaunchKernelGGL(k_moddown_final, dim3(N / EW, l1, 2), dim3(EW), 0, c->stream, acc, (size_t)ext * N, conv,
                     (size_t)l1 * N, k, out, (size_t)l1 * N, add0, g_add0, add1, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

struct RSConst {
  uint64_t h[64];          // floor(q_l / 2) mod q_i
  uint64_t inv[64], inv_s[64];
};

// d_c[i] = (h - ((x_c + h) mod q_l)) mod q_i, x_c = last limb in coefficient form
__global__ void k_rescale_prep(const uint64_t* __restrict__ last, uint64_t* __restrict__ d, int lvl, uint64_t hl,
                               RSConst k, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const uint64_t ql = mods[lvl].q, q = mods[i].q;
  uint64_t y = add_mod(last[c * N + j], hl, ql);   // < q_l < q_i (descending chain)
  d[(c * lvl + i) * N + j] = sub_mod(k.h[i], y, q);
}

// c'_i = (c_i + d_i) * q_l^-1, compacted from [2][l+1][N] to [2][l][N]; one thread per (j, c)
__global__ void k_rescale_final(uint64_t* __restrict__ ct, const uint64_t* __restrict__ d, int lvl, RSConst k,
                                int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int c = blockIdx.y;
  for (int i = 0; i < lvl; ++i) {
    const uint64_t q = mods[i].q;
    uint64_t v = add_mod(ct[(c * (lvl + 1) + i) * N + j], d[(c * lvl + i) * N + j], q);
    ct[(c * lvl + i) * N + j] = mul_shoup(v, k.inv[i], k.inv_s[i], q);
  }
}

void rescale_inplace(ckks_ctx* c, uint64_t* ct, int level) {
  if (level < 1) FICGCN_THROW(ELEVEL_, "rescale at level 0");
  if (level > 63) FICGCN_THROW(EINVAL_, "too many primes");
  const size_t N = c->N;
  const int l1 = level + 1;
  uint64_t* last = (uint64_t*)c->buf(S_RS_TMP, 2 * N * 8);
  HIPCHECK(hipMemcpyAsync(last, ct + (size_t)level * N, N * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHECK(hipMemcpyAsync(last + N, ct + (size_t)(l1 + level) * N, N * 8, hipMemcpyDeviceToDevice, c->stream));
  ntt_inv(c, last, 1, LimbMap{level, 1 << 30, 0}, 2, N);
  RSConst k{};
  uint64_t ql = c->mod[level], hl = ql / 2;
  for (int i = 0; i < level; ++i) {
    uint64_t q = c->mod[i];
    k.h[i] = hl % q;
    k.inv[i] = invmod(ql % q, q);
    k.inv_s[i] = shoup(k.inv[i], q);
  }
  uint64_t* d = (uint64_t*)c->buf(S_RS_D, (size_t)2 * level * N * 8);
  hipLaunchKernelGGL(k_rescale_prep, dim3(N / EW, level, 2), dim3(EW), 0, c->stream, last, d, level, hl, k, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
  ntt_fwd(c, d, level, lm_q(level), 2, (size_t)level * N);
  hipLaunchKernelGGL(k_rescale_final, dim3(N / EW, 2), dim3(EW), 0, c->stream, ct, d, level, k, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

// d0 = x0 y0, d1 = x0 y1 + x1 y0, d2 = x1 y1 ; d is [3][l+1][N]
__global__ void k_tensor(const uint64_t* __restrict__ x, const uint64_t* __restrict__ y, uint64_t* __restrict__ d,
                         int l1, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y;
  const Mod m = mods[i];
  const size_t o0 = i * N + j, o1 = (l1 + i) * N + j;
  uint64_t x0 = x[o0], x1 = x[o1], y0 = y[o0], y1 = y[o1];
  d[o0] = reduce128((u128)x0 * y0, m);
  d[o1] = reduce128((u128)x0 * y1 + (u128)x1 * y0, m);
  d[(2 * l1 + i) * N + j] = reduce128((u128)x1 * y1, m);
}

void tensor(ckks_ctx* c, const uint64_t* x, const uint64_t* y, uint64_t* d, int level) {
  hipLaunchKernelGGL(k_tensor, dim3(c->N / EW, level + 1), dim3(EW), 0, c->stream, x, y, d, level + 1, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
}

__global__ void k_mac_ext(uint64_t* __restrict__ A, const uint64_t* __restrict__ acc, const uint64_t* __restrict__ pt,
                          int ext, int l1, int L, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y, c = blockIdx.z;
  const Mod m = mods[i < l1 ? i : i - l1 + L];
  const size_t o = ((size_t)c * ext + i) * N + j;
  A[o] = add_mod(A[o], pt ? reduce128((u128)acc[o] * pt[(size_t)i * N + j], m) : acc[o], m.q);
}

void mac_ext(ckks_ctx* c, uint64_t* A, const uint64_t* acc, const uint64_t* pt, int level) {
  const int l1 = level + 1, ext = l1 + c->alpha;
  hipLaunchKernelGGL(k_mac_ext, dim3(c->N / EW, ext, 2), dim3(EW), 0, c->stream, A, acc, pt, ext, l1, c->L, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
}

void copy_d2d(ckks_ctx* c, void* dst, const void* src, size_t bytes) {
  HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
}

__global__ void k_ew_mul(uint64_t* __restrict__ out, const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                         LimbMap map, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y;
  const Mod m = mods[lm_mod(map, i)];
  out[i * N + j] = reduce128((u128)a[i * N + j] * b[i * N + j], m);
}

void ew_mul(ckks_ctx* c, uint64_t* out, const uint64_t* a, const uint64_t* b, int n_limbs, LimbMap map) {
  hipLaunchKernelGGL(k_ew_mul, dim3(c->N / EW, n_limbs), dim3(EW), 0, c->stream, out, a, b, map, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
}

// m = c0 + c1 * s over q_0..q_l
__global__ void k_decrypt(const uint64_t* __restrict__ ct, const uint64_t* __restrict__ s, int l1, int log_n,
                          const Mod* __restrict__ mods, uint64_t* __restrict__ m) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)EW + threadIdx.x;
  const int i = blockIdx.y;
  const Mod md = mods[i];
  m[i * N + j] = add_mod(ct[i * N + j], reduce128((u128)ct[(l1 + i) * N + j] * s[i * N + j], md), md.q);
}

void decrypt_core(ckks_ctx* c, const uint64_t* ct, const uint64_t* s_ntt, int level, uint64_t* m) {
  hipLaunchKernelGGL(k_decrypt, dim3(c->N / EW, level + 1), dim3(EW), 0, c->stream, ct, s_ntt, level + 1, c->log_n,
                     c->t.mods, m);
  HIPCHECK(hipGetLastError());
}

}  // namespace ficgcn
