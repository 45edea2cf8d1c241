/*
 * Oracle core: plain, exact CPU arithmetic for RNS-CKKS.  TEST INFRASTRUCTURE
 * ONLY -- used by the test-suite, the smoke check and the CPU baseline; the
 * GPU library never links or calls it.
 *
 * Everything here is the textbook definition written out with 128-bit
 * intermediate products (no lazy reduction, no precomputed quotients):
 *   - ring R_q = Z_q[X]/(X^N + 1) of the CKKS scheme (paper Sec. 2.1);
 *   - the negacyclic NTT evaluates a(X) at the odd powers psi^(2i+1) of a
 *     primitive 2N-th root psi, in natural order (an internal representation:
 *     every public result is in coefficient form);
 *   - the Galois automorphism X -> X^g on coefficients;
 *   - fast base conversion sum_i [x_i * (B/b_i)^-1]_{b_i} * (B/b_i) mod p;
 *   - the ChaCha20 block function of RFC 8439 (randomness of keys/ciphertexts).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
/* a, b in [0, q) with q < 2^63 */
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }

uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = or_mulmod(r, a, q);
    a = or_mulmod(a, a, q);
    e >>= 1;
  }
  return r;
}

/* ---------------- elementwise vectors mod q ---------------- */
void or_vec_mul(const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) out[i] = or_mulmod(a[i], b[i], q);
}
void or_vec_add(const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) out[i] = addmod(a[i], b[i], q);
}
void or_vec_sub(const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) out[i] = submod(a[i], b[i], q);
}
void or_vec_scale(const uint64_t* a, uint64_t c, uint64_t* out, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) out[i] = or_mulmod(a[i], c, q);
}
/* out[i] = a[i] mod q for arbitrary 64-bit a */
void or_vec_reduce(const uint64_t* a, uint64_t* out, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) out[i] = a[i] % q;
}
/* signed small integers -> residues */
void or_vec_from_signed(const int64_t* a, uint64_t* out, size_t n, uint64_t q) {
  for (size_t i = 0; i < n; ++i) {
    int64_t v = a[i];
    uint64_t m = (uint64_t)(v < 0 ? -(v + 1) : v) % q;   /* |v| or |v|-1, no overflow */
    if (v < 0) m = submod(0, (m + 1) % q, q);
    out[i] = m;
  }
}

/* ---------------- negacyclic NTT (natural order) ---------------- */
static void bit_reverse(uint64_t* a, size_t n) {
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
  }
}

/* cyclic DFT over Z_q with root w of order n: A[k] = sum_j a[j] w^(jk) */
static void cyclic_dft(uint64_t* a, size_t n, uint64_t q, uint64_t w) {
  bit_reverse(a, n);
  for (size_t len = 2; len <= n; len <<= 1) {
    uint64_t wl = or_powmod(w, n / len, q);
    for (size_t i = 0; i < n; i += len) {
      uint64_t x = 1;
      for (size_t j = 0; j < len / 2; ++j) {
        uint64_t u = a[i + j], v = or_mulmod(a[i + j + len / 2], x, q);
        a[i + j] = addmod(u, v, q);
        a[i + j + len / 2] = submod(u, v, q);
        x = or_mulmod(x, wl, q);
      }
    }
  }
}

/* a <- (a(psi^1), a(psi^3), ..., a(psi^(2N-1))) */
void or_ntt_fwd(uint64_t* a, size_t n, uint64_t q, uint64_t psi) {
  uint64_t x = 1;
  for (size_t j = 0; j < n; ++j) { a[j] = or_mulmod(a[j], x, q); x = or_mulmod(x, psi, q); }
  cyclic_dft(a, n, q, or_mulmod(psi, psi, q));
}

/* inverse of or_ntt_fwd */
void or_ntt_inv(uint64_t* a, size_t n, uint64_t q, uint64_t psi) {
  uint64_t psi_inv = or_powmod(psi, q - 2, q);
  cyclic_dft(a, n, q, or_mulmod(psi_inv, psi_inv, q));
  uint64_t n_inv = or_powmod(n % q, q - 2, q);
  uint64_t x = n_inv;
  for (size_t j = 0; j < n; ++j) { a[j] = or_mulmod(a[j], x, q); x = or_mulmod(x, psi_inv, q); }
}

/* out = a * b in Z_q[X]/(X^N+1) (coefficient form in and out) */
void or_negacyclic_mul(const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n, uint64_t q, uint64_t psi) {
  uint64_t* fa = (uint64_t*)malloc(n * 8);
  uint64_t* fb = (uint64_t*)malloc(n * 8);
  memcpy(fa, a, n * 8);
  memcpy(fb, b, n * 8);
  or_ntt_fwd(fa, n, q, psi);
  or_ntt_fwd(fb, n, q, psi);
  for (size_t i = 0; i < n; ++i) fa[i] = or_mulmod(fa[i], fb[i], q);
  or_ntt_inv(fa, n, q, psi);
  memcpy(out, fa, n * 8);
  free(fa);
  free(fb);
}

/* schoolbook negacyclic product, O(N^2): the definition itself */
void or_negacyclic_mul_naive(const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n, uint64_t q) {
  for (size_t k = 0; k < n; ++k) out[k] = 0;
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j) {
      uint64_t p = or_mulmod(a[i], b[j], q);
      size_t k = i + j;
      if (k < n) out[k] = addmod(out[k], p, q);
      else out[k - n] = submod(out[k - n], p, q);
    }
}

/* ---------------- Galois automorphism X -> X^g (g odd) ---------------- */
void or_automorph(const uint64_t* in, uint64_t* out, size_t n, uint64_t g, uint64_t q) {
  size_t two_n = 2 * n;
  for (size_t i = 0; i < n; ++i) {
    size_t k = (size_t)(((u128)i * g) % two_n);
    if (k < n) out[k] = in[i];
    else out[k - n] = submod(0, in[i], q);
  }
}

/* ---------------- fast base conversion ----------------
 * in:  ks rows of n residues (row i modulo src[i])
 * out: n residues modulo p of  sum_i [in_i * hat_inv[i]]_{src_i} * hat_mod_p[i]
 * where hat_inv[i] = (B/src_i)^-1 mod src_i and hat_mod_p[i] = (B/src_i) mod p.
 */
void or_fast_bconv(const uint64_t* in, size_t n, const uint64_t* src, size_t ks,
                   const uint64_t* hat_inv, const uint64_t* hat_mod_p, uint64_t p, uint64_t* out) {
  for (size_t j = 0; j < n; ++j) {
    uint64_t acc = 0;
    for (size_t i = 0; i < ks; ++i) {
      uint64_t y = or_mulmod(in[i * n + j], hat_inv[i], src[i]);
      acc = addmod(acc, or_mulmod(y % p, hat_mod_p[i], p), p);
    }
    out[j] = acc;
  }
}

/* ---------------- ChaCha20 block function (RFC 8439, Sec. 2.3) ---------------- */
static uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }
#define QR(a, b, c, d)                 \
  a += b; d ^= a; d = rotl32(d, 16);   \
  c += d; b ^= c; b = rotl32(b, 12);   \
  a += b; d ^= a; d = rotl32(d, 8);    \
  c += d; b ^= c; b = rotl32(b, 7);

void or_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]) {
  uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                    key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                    counter, nonce[0], nonce[1], nonce[2]};
  uint32_t x[16];
  memcpy(x, s, sizeof x);
  for (int i = 0; i < 10; ++i) {
    QR(x[0], x[4], x[8], x[12]) QR(x[1], x[5], x[9], x[13]) QR(x[2], x[6], x[10], x[14]) QR(x[3], x[7], x[11], x[15])
    QR(x[0], x[5], x[10], x[15]) QR(x[1], x[6], x[11], x[12]) QR(x[2], x[7], x[8], x[13]) QR(x[3], x[4], x[9], x[14])
  }
  for (int i = 0; i < 16; ++i) out[i] = x[i] + s[i];
}

/* nblocks consecutive blocks starting at counter `first` -> out[16*nblocks] */
void or_chacha20_stream(const uint32_t key[8], const uint32_t nonce[3], uint32_t first, size_t nblocks, uint32_t* out) {
  for (size_t b = 0; b < nblocks; ++b) or_chacha20_block(key, first + (uint32_t)b, nonce, out + 16 * b);
}

/* ---------------- sampler helper ----------------
 * out[j] = (w[4j] + w[4j+1]*2^32 + w[4j+2]*2^64 + w[4j+3]*2^96) mod q
 */
void or_uniform_from_words(const uint32_t* w, size_t n, uint64_t q, uint64_t* out) {
  for (size_t j = 0; j < n; ++j) {
    u128 x = ((u128)w[4 * j + 3] << 96) | ((u128)w[4 * j + 2] << 64) | ((u128)w[4 * j + 1] << 32) | (u128)w[4 * j];
    out[j] = (uint64_t)(x % q);
  }
}
