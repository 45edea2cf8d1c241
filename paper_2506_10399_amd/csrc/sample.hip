// Randomness, key generation and symmetric encryption on the device.
//
// Every random polynomial is read from a ChaCha20 stream (block function of
// RFC 8439): key words (seed mod 2^32, seed >> 32, 0, 0, 0, 0, 0, 0), a
// three-word nonce naming the stream, block counter 0, 1, ...  Coefficient j
//   uniform mod q : words 4j..4j+3 as a little-endian 128-bit integer, mod q
//   ternary       : x = words 2j, 2j+1 as a 64-bit integer, (x mod 3) - 1
//   CBD(21)       : popcount(x & (2^21-1)) - popcount((x >> 21) & (2^21-1))
// Streams: secret (1,0,0); key 'a' (2, tag, digit*65536 + prime index);
// key 'e' (3, tag, digit); ciphertext 'a' (4, id, prime index); ciphertext
// 'e' (5, id, 0).  A ciphertext's 'a' may be keyed by a public seed of its own
// (a seeded ciphertext: the server regenerates 'a' from that seed and the id).  A rotation key's tag is its Galois element, the
// relinearisation key's tag is 0.
#include <algorithm>

#include "internal.h"

namespace ficgcn {

constexpr int SB = 256;

__device__ __forceinline__ uint32_t rotl(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

__device__ __forceinline__ void qr(uint32_t& a, uint32_t& b, uint32_t& c, uint32_t& d) {
  a += b; d ^= a; d = rotl(d, 16);
  c += d; b ^= c; b = rotl(b, 12);
  a += b; d ^= a; d = rotl(d, 8);
  c += d; b ^= c; b = rotl(b, 7);
}

__device__ void chacha_block(uint64_t seed, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t ctr, uint32_t out[16]) {
  uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, (uint32_t)seed, (uint32_t)(seed >> 32),
                    0, 0, 0, 0, 0, 0, ctr, n0, n1, n2};
  uint32_t x[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = s[i];
#pragma unroll 1
  for (int r = 0; r < 10; ++r) {
    qr(x[0], x[4], x[8], x[12]); qr(x[1], x[5], x[9], x[13]); qr(x[2], x[6], x[10], x[14]); qr(x[3], x[7], x[11], x[15]);
    qr(x[0], x[5], x[10], x[15]); qr(x[1], x[6], x[11], x[12]); qr(x[2], x[7], x[8], x[13]); qr(x[3], x[4], x[9], x[14]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

// one thread = one block = 4 coefficients of one limb; blockIdx.z = polynomial
// z at out + z * poly_stride, drawn from the stream with nonce word a + z
__global__ void k_uniform(uint64_t* __restrict__ out, uint64_t seed, uint32_t kind, uint32_t a, uint32_t b0,
                          LimbMap map, int log_n, const Mod* __restrict__ mods, size_t poly_stride) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t blk = blockIdx.x * SB + threadIdx.x;
  if ((size_t)blk * 4 >= N) return;
  const int i = blockIdx.y;
  const int mi = lm_mod(map, i);
  out += blockIdx.z * poly_stride;
  uint32_t w[16];
  chacha_block(seed, kind, a + blockIdx.z, b0 + (uint32_t)mi, blk, w);
  const Mod m = mods[mi];
  for (int u = 0; u < 4; ++u) {
    uint64_t lo = (uint64_t)w[4 * u] | ((uint64_t)w[4 * u + 1] << 32);
    uint64_t hi = (uint64_t)w[4 * u + 2] | ((uint64_t)w[4 * u + 3] << 32);
    out[i * N + (size_t)blk * 4 + u] = reduce128(hi, lo, m);
  }
}

void sample_uniform(ckks_ctx* c, uint64_t* out, uint64_t seed, uint32_t kind, uint32_t a, uint32_t b0, int n_limbs,
                    LimbMap map, uint32_t) {
  int nb = (c->N / 4 + SB - 1) / SB;
  hipLaunchKernelGGL(k_uniform, dim3(nb, n_limbs), dim3(SB), 0, c->stream, out, seed, kind, a, b0, map, c->log_n,
                     c->t.mods, (size_t)0);
  HIPCHECK(hipGetLastError());
}

void expand_seeded(ckks_ctx* c, uint64_t a_seed, uint32_t ct_id0, size_t count, int level, uint64_t* cts) {
  const size_t N = c->N;
  const int l1 = level + 1;
  const size_t ct_words = 2 * (size_t)l1 * N;
  const int nb = (int)((N / 4 + SB - 1) / SB);
  constexpr size_t CHUNK = 4096;   // polynomials per launch (grid z)
  for (size_t z0 = 0; z0 < count; z0 += CHUNK) {
    const size_t nz = std::min(CHUNK, count - z0);
    uint64_t* c1 = cts + z0 * ct_words + (size_t)l1 * N;
    hipLaunchKernelGGL(k_uniform, dim3(nb, l1, (uint32_t)nz), dim3(SB), 0, c->stream, c1, a_seed, 4u,
                       ct_id0 + (uint32_t)z0, 0u, lm_q(l1), c->log_n, c->t.mods, ct_words);
    HIPCHECK(hipGetLastError());
    ntt_fwd(c, c1, l1, lm_q(l1), (int)nz, ct_words);
  }
}

// ---- bit-packed residues (transport of client words) ----
// A limb of N residues below 2^bits travels as N * bits / 64 words: residue r of the
// limb holds bits r * bits .. r * bits + bits - 1 of the limb's little-endian bit stream.
// count polynomials of n_limbs limbs: polynomial z's limbs at in + z * in_stride
// (resp. out + z * out_stride), limbs N (packed: N * bits / 64) words apart.

// one thread per packed word: the residues that overlap it, shifted into place
__global__ void k_pack(const uint64_t* __restrict__ in, size_t in_stride, uint64_t* __restrict__ out,
                       size_t out_stride, int bits, int log_n) {
  const size_t N = (size_t)1 << log_n;
  const size_t wpl = (N * (size_t)bits) >> 6;
  const size_t w = blockIdx.x * (size_t)SB + threadIdx.x;
  if (w >= wpl) return;
  const uint64_t* src = in + blockIdx.z * in_stride + (size_t)blockIdx.y * N;
  const uint64_t mask = bits == 64 ? ~0ull : (1ull << bits) - 1;
  const size_t b0 = w * 64;
  uint64_t v = 0;
  for (size_t r = b0 / bits; r < N && r * bits < b0 + 64; ++r) {
    const uint64_t x = src[r] & mask;
    const long long off = (long long)(r * bits) - (long long)b0;   // in (-bits, 64)
    v |= off >= 0 ? x << off : x >> (-off);
  }
  out[blockIdx.z * out_stride + (size_t)blockIdx.y * wpl + w] = v;
}

// one thread per residue: one or two packed words
__global__ void k_unpack(const uint64_t* __restrict__ in, size_t in_stride, uint64_t* __restrict__ out,
                         size_t out_stride, int bits, int log_n) {
  const size_t N = (size_t)1 << log_n;
  const size_t wpl = (N * (size_t)bits) >> 6;
  const size_t r = blockIdx.x * (size_t)SB + threadIdx.x;
  if (r >= N) return;
  const uint64_t* src = in + blockIdx.z * in_stride + (size_t)blockIdx.y * wpl;
  const size_t b = r * bits, w = b >> 6;
  const int sh = (int)(b & 63);
  uint64_t v = src[w] >> sh;
  if (sh + bits > 64) v |= src[w + 1] << (64 - sh);   // the residue's last bit lies in the limb
  const uint64_t mask = bits == 64 ? ~0ull : (1ull << bits) - 1;
  out[blockIdx.z * out_stride + (size_t)blockIdx.y * N + r] = v & mask;
}

void pack_residues(ckks_ctx* c, const uint64_t* in, size_t in_stride, uint64_t* out, size_t out_stride,
                   int n_limbs, size_t count, int bits, bool unpack) {
  const size_t N = c->N;
  const size_t wpl = (N * (size_t)bits) >> 6;
  const size_t units = unpack ? N : wpl;
  const int nb = (int)((units + SB - 1) / SB);
  constexpr size_t CHUNK = 4096;   // polynomials per launch (grid z)
  for (size_t z0 = 0; z0 < count; z0 += CHUNK) {
    const size_t nz = std::min(CHUNK, count - z0);
    if (unpack)
      hipLaunchKernelGGL(k_unpack, dim3(nb, n_limbs, (uint32_t)nz), dim3(SB), 0, c->stream, in + z0 * in_stride,
                         in_stride, out + z0 * out_stride, out_stride, bits, c->log_n);
    else
      hipLaunchKernelGGL(k_pack, dim3(nb, n_limbs, (uint32_t)nz), dim3(SB), 0, c->stream, in + z0 * in_stride,
                         in_stride, out + z0 * out_stride, out_stride, bits, c->log_n);
    HIPCHECK(hipGetLastError());
  }
}

// one thread = one block = 8 coefficients, written as residues of every limb
__global__ void k_small(uint64_t* __restrict__ out, uint64_t seed, uint32_t kind, uint32_t a, uint32_t b, int dist,
                        int n_limbs, LimbMap map, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const uint32_t blk = blockIdx.x * SB + threadIdx.x;
  if ((size_t)blk * 8 >= N) return;
  uint32_t w[16];
  chacha_block(seed, kind, a, b, blk, w);
  for (int u = 0; u < 8; ++u) {
    uint64_t x = (uint64_t)w[2 * u] | ((uint64_t)w[2 * u + 1] << 32);
    int64_t v;
    if (dist == 0) {
      v = (int64_t)(x % 3) - 1;
    } else {
      const uint64_t msk = (1ull << 21) - 1;
      v = (int64_t)__popcll(x & msk) - (int64_t)__popcll((x >> 21) & msk);
    }
    for (int i = 0; i < n_limbs; ++i) {
      uint64_t q = mods[lm_mod(map, i)].q;
      out[i * N + (size_t)blk * 8 + u] = v >= 0 ? (uint64_t)v : q - (uint64_t)(-v);
    }
  }
}

void sample_small_rns(ckks_ctx* c, uint64_t* out, uint64_t seed, uint32_t kind, uint32_t a, uint32_t b, int dist,
                      int n_limbs, LimbMap map) {
  int nb = (c->N / 8 + SB - 1) / SB;
  hipLaunchKernelGGL(k_small, dim3(nb), dim3(SB), 0, c->stream, out, seed, kind, a, b, dist, n_limbs, map, c->log_n,
                     c->t.mods);
  HIPCHECK(hipGetLastError());
}

// b_i = e_i - a_i s_i + [i in digit] (P mod q_i) s'_i   (evaluation form)
__global__ void k_keyb(uint64_t* __restrict__ b, const uint64_t* __restrict__ a, const uint64_t* __restrict__ s,
                       const uint64_t* __restrict__ sp, int d_lo, int d_hi, const uint64_t* __restrict__ pmod,
                       int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)SB + threadIdx.x;
  const int i = blockIdx.y;
  const Mod m = mods[i];
  const size_t o = i * N + j;
  uint64_t v = sub_mod(b[o], reduce128((u128)a[o] * s[o], m), m.q);
  if (i >= d_lo && i < d_hi) v = add_mod(v, reduce128((u128)pmod[i] * sp[o], m), m.q);
  b[o] = v;
}

void keygen_swk(ckks_ctx* c, uint64_t seed, const uint64_t* s_ntt, const uint64_t* sp_ntt, uint64_t tag,
                uint64_t* key) {
  const size_t N = c->N;
  const int nm = c->n_mod();
  const LimbMap full = lm_q(nm);
  // P mod q_i for every Q prime
  std::vector<uint64_t> pm(nm, 0);
  for (int i = 0; i < c->L; ++i) {
    uint64_t v = 1;
    for (int k = 0; k < c->alpha; ++k) v = (uint64_t)((u128)v * (c->mod[c->L + k] % c->mod[i]) % c->mod[i]);
    pm[i] = v;
  }
  uint64_t* pmd = (uint64_t*)c->buf(10, nm * 8);
  HIPCHECK(hipMemcpyAsync(pmd, pm.data(), nm * 8, hipMemcpyHostToDevice, c->stream));
  for (int d = 0; d < c->beta(); ++d) {
    uint64_t* kb = key + ((size_t)d * 2 + 0) * nm * N;
    uint64_t* ka = key + ((size_t)d * 2 + 1) * nm * N;
    sample_uniform(c, ka, seed, 2, (uint32_t)tag, (uint32_t)d * 65536u, nm, full, 0);
    ntt_fwd(c, ka, nm, full, 1, 0);
    sample_small_rns(c, kb, seed, 3, (uint32_t)tag, (uint32_t)d, 1, nm, full);
    ntt_fwd(c, kb, nm, full, 1, 0);
    int lo = d * c->alpha, hi = std::min((d + 1) * c->alpha, c->L);
    hipLaunchKernelGGL(k_keyb, dim3(N / SB, nm), dim3(SB), 0, c->stream, kb, ka, s_ntt, sp_ntt, lo, hi, pmd,
                       c->log_n, c->t.mods);
    HIPCHECK(hipGetLastError());
  }
  // pm lives on the host stack: finish the upload before returning
  HIPCHECK(hipStreamSynchronize(c->stream));
}

// c0 = e - a s + m
__global__ void k_enc(uint64_t* __restrict__ c0, const uint64_t* __restrict__ a, const uint64_t* __restrict__ s,
                      const uint64_t* __restrict__ m, int log_n, const Mod* __restrict__ mods) {
  const size_t N = (size_t)1 << log_n;
  const size_t j = blockIdx.x * (size_t)SB + threadIdx.x;
  const int i = blockIdx.y;
  const Mod md = mods[i];
  const size_t o = i * N + j;
  uint64_t v = sub_mod(c0[o], reduce128((u128)a[o] * s[o], md), md.q);
  c0[o] = add_mod(v, m[o], md.q);
}

void encrypt_sym(ckks_ctx* c, const uint64_t* s_ntt, const uint64_t* m_ntt, int level, uint64_t seed, uint64_t a_seed,
                 uint32_t ct_id, uint64_t* ct) {
  const size_t N = c->N;
  const int l1 = level + 1;
  uint64_t* c0 = ct;
  uint64_t* c1 = ct + (size_t)l1 * N;
  expand_seeded(c, a_seed, ct_id, 1, level, ct);
  sample_small_rns(c, c0, seed, 5, ct_id, 0, 1, l1, lm_q(l1));
  ntt_fwd(c, c0, l1, lm_q(l1), 1, 0);
  hipLaunchKernelGGL(k_enc, dim3(N / SB, l1), dim3(SB), 0, c->stream, c0, c1, s_ntt, m_ntt, c->log_n, c->t.mods);
  HIPCHECK(hipGetLastError());
}

}  // namespace ficgcn
