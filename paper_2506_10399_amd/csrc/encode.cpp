// Canonical-embedding tables and decode (host, FP64).
//
// Slot j of m(X) in Z[X]/(X^N+1) is m(zeta^(5^j)), zeta = exp(i pi / N); the
// conjugate slots sit at zeta^(-5^j).  Encoding (on the device, from the
// tables built here) evaluates the inverse embedding with one complex FFT
// over the N odd powers of zeta:
//   v_s = value at zeta^(2s+1),  m_i = Re(exp(-i pi i / N) FFT(v)_i) / N,
// then rounds half-to-even after scaling.  Decoding CRT-lifts each
// coefficient exactly (multi-word integers), centres it, divides by the scale
// and evaluates the embedding with the inverse FFT.
#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace ficgcn {

typedef std::complex<double> cd;

// exp(-2 pi i k / n) for k < n/2, and exp(-i pi i / n) for i < n; cached per n
struct FftTables {
  std::vector<cd> root, twist;
};

static const FftTables& tables(size_t n) {
  static std::mutex mu;
  static std::map<size_t, FftTables> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(n);
  if (it != cache.end()) return it->second;
  FftTables t;
  t.root.resize(n / 2);
  for (size_t k = 0; k < n / 2; ++k) t.root[k] = cd(std::cos(2 * M_PI * k / n), -std::sin(2 * M_PI * k / n));
  t.twist.resize(n);
  for (size_t i = 0; i < n; ++i) t.twist[i] = cd(std::cos(M_PI * i / n), -std::sin(M_PI * i / n));
  return cache[n] = t;
}

// (a.re c.re - a.im c.im, a.re c.im + a.im c.re): the product std::complex
// computes for finite values, without its out-of-line NaN/infinity handling
static inline cd cmul(cd a, cd c) {
  return cd(a.real() * c.real() - a.imag() * c.imag(), a.real() * c.imag() + a.imag() * c.real());
}

static void fft(std::vector<cd>& a, bool inverse, const FftTables& T) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t step = n / len;
    for (size_t i = 0; i < n; i += len) {
      for (size_t k = 0; k < len / 2; ++k) {
        cd w = T.root[k * step];
        if (inverse) w = std::conj(w);
        cd u = a[i + k], v = cmul(a[i + k + len / 2], w);
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
    }
  }
}

// 5^j mod 2N for the N/2 slots, cached per N
static const std::vector<uint32_t>& slot_exponents(int N) {
  static std::mutex mu;
  static std::map<int, std::vector<uint32_t>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(N);
  if (it != cache.end()) return it->second;
  std::vector<uint32_t> r(N / 2);
  uint64_t x = 1;
  for (int j = 0; j < N / 2; ++j) {
    r[j] = (uint32_t)x;
    x = x * 5 % (2 * (uint64_t)N);
  }
  return cache[N] = r;
}

void encode_tables(int N, std::vector<double>& root, std::vector<double>& twist, std::vector<uint32_t>& pos) {
  const FftTables& T = tables(N);
  const std::vector<uint32_t>& r = slot_exponents(N);
  root.resize((size_t)N);
  for (int k = 0; k < N / 2; ++k) {
    root[2 * k] = T.root[k].real();
    root[2 * k + 1] = T.root[k].imag();
  }
  twist.resize((size_t)2 * N);
  for (int i = 0; i < N; ++i) {
    twist[2 * i] = T.twist[i].real();
    twist[2 * i + 1] = T.twist[i].imag();
  }
  pos.resize((size_t)N);
  for (int j = 0; j < N / 2; ++j) {
    pos[2 * j] = (r[j] - 1) / 2;
    pos[2 * j + 1] = ((2 * (uint32_t)N - r[j]) - 1) / 2;
  }
}

void decode_values(int N, const std::vector<double>& m, double scale, double* re, double* im, size_t n) {
  std::vector<cd> w(N);
  const FftTables& T = tables(N);
  for (int i = 0; i < N; ++i) w[i] = cmul(cd(m[i] / scale, 0), std::conj(T.twist[i]));
  fft(w, true, T);
  const std::vector<uint32_t>& r = slot_exponents(N);
  for (size_t j = 0; j < n && j < (size_t)N / 2; ++j) {
    cd z = w[(r[j] - 1) / 2];
    if (re) re[j] = z.real();
    if (im) im[j] = z.imag();
  }
}

// ---- exact CRT lift of residues to a centred double ----
struct Big {
  std::vector<uint64_t> w;   // little-endian words
};

static void big_mul_small_add(Big& acc, const Big& x, uint64_t k) {
  // acc += x * k
  if (acc.w.size() < x.w.size() + 1) acc.w.resize(x.w.size() + 1, 0);
  u128 carry = 0;
  size_t i = 0;
  for (; i < x.w.size(); ++i) {
    u128 t = (u128)x.w[i] * k + acc.w[i] + carry;
    acc.w[i] = (uint64_t)t;
    carry = t >> 64;
  }
  for (; carry && i < acc.w.size(); ++i) {
    u128 t = (u128)acc.w[i] + carry;
    acc.w[i] = (uint64_t)t;
    carry = t >> 64;
  }
  if (carry) acc.w.push_back((uint64_t)carry);
}

static int big_cmp(const Big& a, const Big& b) {
  size_t n = std::max(a.w.size(), b.w.size());
  for (size_t i = n; i-- > 0;) {
    uint64_t x = i < a.w.size() ? a.w[i] : 0, y = i < b.w.size() ? b.w[i] : 0;
    if (x != y) return x < y ? -1 : 1;
  }
  return 0;
}

static void big_sub(Big& a, const Big& b) {   // a -= b, a >= b
  uint64_t borrow = 0;
  for (size_t i = 0; i < a.w.size(); ++i) {
    uint64_t y = i < b.w.size() ? b.w[i] : 0;
    u128 t = (u128)a.w[i] - y - borrow;
    a.w[i] = (uint64_t)t;
    borrow = (uint64_t)(t >> 64) ? 1 : 0;
  }
}

static double big_to_double(const Big& a) {
  double r = 0;
  for (size_t i = a.w.size(); i-- > 0;) r = r * 18446744073709551616.0 + (double)a.w[i];
  return r;
}

// residues [k][N] over mods[0..k) -> centred integers as doubles
void crt_center(const std::vector<uint64_t>& mods, const uint64_t* res, int N, std::vector<double>& out) {
  const int k = (int)mods.size();
  Big Q;
  Q.w = {1};
  for (uint64_t q : mods) {
    Big t;
    big_mul_small_add(t, Q, q);
    Q = t;
  }
  std::vector<Big> hat(k);
  std::vector<uint64_t> hinv(k), hinv_s(k);
  for (int i = 0; i < k; ++i) {
    Big h;
    h.w = {1};
    uint64_t hm = 1;
    for (int u = 0; u < k; ++u)
      if (u != i) {
        Big t;
        big_mul_small_add(t, h, mods[u]);
        h = t;
        hm = (uint64_t)((u128)hm * (mods[u] % mods[i]) % mods[i]);
      }
    hat[i] = h;
    hinv[i] = invmod(hm, mods[i]);
    hinv_s[i] = shoup(hinv[i], mods[i]);
  }
  Big halfQ;   // floor(Q / 2)
  halfQ.w = Q.w;
  for (size_t i = 0; i < halfQ.w.size(); ++i) {
    halfQ.w[i] >>= 1;
    if (i + 1 < halfQ.w.size()) halfQ.w[i] |= Q.w[i + 1] << 63;
  }
  out.resize(N);
  for (int j = 0; j < N; ++j) {
    Big s;
    s.w.assign(Q.w.size() + 1, 0);
    for (int i = 0; i < k; ++i) {
      uint64_t y = mul_shoup(res[(size_t)i * N + j], hinv[i], hinv_s[i], mods[i]);
      big_mul_small_add(s, hat[i], y);
    }
    while (big_cmp(s, Q) >= 0) big_sub(s, Q);
    if (big_cmp(s, halfQ) > 0) {
      Big t = Q;
      t.w.resize(s.w.size(), 0);
      big_sub(t, s);
      out[j] = -big_to_double(t);
    } else {
      out[j] = big_to_double(s);
    }
  }
}

}  // namespace ficgcn
