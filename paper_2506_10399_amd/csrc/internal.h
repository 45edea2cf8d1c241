// Internal declarations of the FicGCN MI355X library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "modarith.h"

namespace ficgcn {

// Status codes mirror include/ficgcn.h.
enum { OK = 0, EINVAL_ = -1, ELEVEL_ = -2, ESCALE_ = -3, ENOKEY_ = -4, ENOMEM_ = -5, EDEVICE_ = -6, EPLAN_ = -7 };

struct Error {
  int code;
  std::string msg;
};

void set_error(const std::string& msg);
#define FICGCN_THROW(code, msg) throw ::ficgcn::Error{(code), (msg)}
#define HIPCHECK(x)                                                                                 \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) FICGCN_THROW(::ficgcn::EDEVICE_, std::string(#x) + ": " + hipGetErrorString(e_));   \
  } while (0)

// Modulus index of limb i of a polynomial: j = i + first; j < split ? j : j + pofs.
// Q primes are indices 0..L-1, special primes L..L+alpha-1.
struct LimbMap {
  int first, split, pofs;
};
FICGCN_FD int lm_mod(const LimbMap& m, int i) {
  int j = i + m.first;
  return j < m.split ? j : j + m.pofs;
}
inline LimbMap lm_q(int n) { return LimbMap{0, n, 0}; }                     // plain Q limbs 0..n-1
inline LimbMap lm_ext(int level, int L) { return LimbMap{0, level + 1, L - level - 1}; }  // Q_l then P

// Device-resident per-modulus tables.
struct Tables {
  uint64_t* psi = nullptr;     // [n_mod][N] psi^{brev(k)}
  uint64_t* psi_s = nullptr;   // Shoup companions
  uint64_t* ipsi = nullptr;    // [n_mod][N] psi^{-brev(k)}
  uint64_t* ipsi_s = nullptr;
  double* psi_f = nullptr;     // [n_mod][N] the same twiddles as doubles (exact below 2^53)
  double* ipsi_f = nullptr;
  Mod* mods = nullptr;         // [n_mod]
  uint64_t* ninv = nullptr;    // [n_mod] N^{-1}
  uint64_t* ninv_s = nullptr;
};

// Fast base conversion constants from a source prime set to a destination set.
struct BConv {
  int n_src = 0, n_dst = 0;
  std::vector<int> src, dst;     // modulus indices
  uint64_t* dev = nullptr;       // [n_src] hat_inv, [n_src] hat_inv_shoup, [n_dst][n_src] hat_mod_dst
  int* idx = nullptr;            // [n_src] source modulus indices, then [n_dst] destination indices
};

}  // namespace ficgcn

namespace ficgcn {
// Device buffers of one recorded launch sequence (a layer captured in a HIP
// graph).  RECORD: every table upload and scratch request gets a buffer of
// its own, kept in call order; REPLAY: the same calls get the same buffers
// back in the same order, with no upload and no host synchronisation, so
// the sequence can be captured.
struct Recorder {
  enum Mode { RECORD, REPLAY } mode = RECORD;
  std::vector<std::pair<void*, size_t>> bufs;
  size_t cursor = 0;
  ~Recorder();
};
}  // namespace ficgcn

struct ckks_ctx {
  int log_n = 0, N = 0, L = 0, alpha = 0, log_scale = 40, q_bits = 0, p_bits = 0;
  ficgcn::Recorder* rec = nullptr;   // set while a layer is recorded or captured
  std::vector<uint64_t> mod;         // Q primes (descending) then P primes
  std::vector<uint64_t> psi;         // primitive 2N-th root per modulus
  ficgcn::Tables t;                  // device copies, uploaded on first device use
  std::vector<uint64_t> h_psi, h_psi_s, h_ipsi, h_ipsi_s, h_ninv, h_ninv_s;   // host tables
  std::vector<ficgcn::Mod> h_mods;
  bool on_device = false;
  int ntt_cols[2] = {16, 4};          // NTT workgroup width (column pass, row pass); autotuned
  int ntt_split = 0;                  // log2 of the column pass's transform size (0: log_n / 2); autotuned
  hipStream_t stream = nullptr;
  int device = 0;
  std::map<std::pair<int, int>, ficgcn::BConv> modup;   // (level, digit)
  std::map<int, ficgcn::BConv> moddown;                  // level
  // grow-only scratch buffers by slot: ops.hip 1-9, sample/capi 10-29, gcn.cpp 30-49 and 70-79,
  // ks_batch.hip 50-64 and 80-89, search.cpp 65-66 (a slot's memory moves when it grows, so one
  // user per slot)
  std::vector<std::pair<void*, size_t>> scratch;
  // device tables of the GPU encoder (built on its first use)
  double* enc_root = nullptr;    // [N/2] (re, im)
  double* enc_twist = nullptr;   // [N] (re, im)
  uint32_t* enc_pos = nullptr;   // [N] slot j -> FFT input of the slot and of its conjugate
  int* enc_flag = nullptr;       // set when a coefficient leaves 63 bits
  // kernel timing (HIP events on `stream`), see ficgcn_profile_enable
  bool profiling = false;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof;
  int beta() const { return (L + alpha - 1) / alpha; }
  int n_mod() const { return L + alpha; }
  void* buf(int slot, size_t bytes);
  ~ckks_ctx();
};

struct ckks_keys {
  ckks_ctx* ctx = nullptr;
  bool has_secret = false;
  uint64_t seed = 0;                         // key generation seed (client object only)
  uint64_t* s_ntt = nullptr;                 // [L+alpha][N] secret in NTT form (client object only)
  std::map<uint64_t, uint64_t*> swk;         // tag -> [beta][2][L+alpha][N] NTT form (tag 0 = relin)
  ~ckks_keys();
};

namespace ficgcn {

// Records a start/stop event pair around the enclosed launches when the
// context is profiling.
struct ProfScope {
  ckks_ctx* c;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(ckks_ctx* cc, const char* n) : c(cc), name(n) {
    if (!c->profiling || c->rec) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(a, c->stream);
  }
  // records the end event now (before a host wait that follows the timed launches)
  void stop() {
    if (!c->profiling || c->rec || !a || !b) return;
    (void)hipEventRecord(b, c->stream);
    c->prof[name].push_back({a, b});
    a = b = nullptr;
  }
  ~ProfScope() { stop(); }
};

// Scratch of `bytes` (context slot, or the recorder's buffer), a device copy
// of a host table (slot + asynchronous copy, or the recorder's buffer), and
// a stream synchronisation that a replay being captured skips.
void* dev_scratch(ckks_ctx* c, int slot, size_t bytes);
void* dev_table(ckks_ctx* c, int slot, const void* host, size_t bytes);
void stream_sync(ckks_ctx* c);

uint64_t powmod(uint64_t a, uint64_t e, uint64_t q);
uint64_t invmod(uint64_t a, uint64_t q);
uint64_t shoup(uint64_t w, uint64_t q);
Mod make_mod(uint64_t q);
void build_context(ckks_ctx* c);
void ensure_device(ckks_ctx* c);   // uploads the tables once (needs a GPU)
const BConv& get_modup(ckks_ctx* c, int level, int digit);
const BConv& get_moddown(ckks_ctx* c, int level);
uint64_t galois_elt(ckks_ctx* c, int64_t step);

// ---- NTT (ntt.hip) ----
// n_polys polynomials, each n_limbs limbs of N words; limb i of poly p at
// base + p*poly_stride + i*N, modulus lm_mod(map, i).  Limbs with
// (skip_alpha > 0 && i < skip_q && i / skip_alpha == p mod ceil(skip_q / skip_alpha))
// are left untouched (the digits' own limbs of one or more ModUp outputs).
void ntt_fwd(ckks_ctx* c, uint64_t* base, int n_limbs, LimbMap map, int n_polys, size_t poly_stride,
             int skip_alpha = 0, int skip_q = 0);
void ntt_inv(ckks_ctx* c, uint64_t* base, int n_limbs, LimbMap map, int n_polys, size_t poly_stride);

// ---- elementwise and key-switching kernels (ops.hip) ----
struct PtrList {
  enum { MAX = 16 };
  const uint64_t* p[MAX];
};
struct OutList {
  enum { MAX = 16 };
  uint64_t* p[MAX];
};
void pmul_acc(ckks_ctx* c, uint64_t* acc, const PtrList& cts, const PtrList& pts, int k, int n_limbs);
void smul_acc(ckks_ctx* c, uint64_t* acc, const PtrList& cts, const uint64_t* consts_dev, int k, int n_limbs);
void add_inplace(ckks_ctx* c, uint64_t* acc, const uint64_t* in, int n_limbs, int n_polys);
void automorph_ntt(ckks_ctx* c, uint64_t* out, const uint64_t* in, uint64_t g, int n_limbs, int n_polys);
void bconv(ckks_ctx* c, const BConv& bc, const uint64_t* src, uint64_t* dst_base, const int* dst_pos_dev,
           int n_polys, size_t src_poly_stride, size_t dst_poly_stride);
// tmp / conv: caller scratch of (level+1) resp. 2 (level+1) limbs, or null for the context's own
void modup(ckks_ctx* c, const uint64_t* a_ntt, int level, uint64_t* D, uint64_t* tmp = nullptr);
void keymac(ckks_ctx* c, uint64_t* acc, const uint64_t* D, const uint64_t* key, int level, uint64_t g);
void moddown(ckks_ctx* c, uint64_t* acc, int level, uint64_t* out, const uint64_t* add0, uint64_t g_add0,
             const uint64_t* add1, uint64_t* conv = nullptr);
void rescale_inplace(ckks_ctx* c, uint64_t* ct, int level);
void tensor(ckks_ctx* c, const uint64_t* x, const uint64_t* y, uint64_t* d, int level);
void copy_d2d(ckks_ctx* c, void* dst, const void* src, size_t bytes);
// A (+)= acc (.) pt over the key basis Q_l then P (both components); pt null: A += acc
void mac_ext(ckks_ctx* c, uint64_t* A, const uint64_t* acc, const uint64_t* pt, int level);
// plaintexts on the key basis: [level+1+alpha][N], Q_l limbs then P, evaluation form
void encode_batch_ext(ckks_ctx* c, const double* re, size_t count, size_t n, double scale, int level, uint64_t* dev);
void pt_load_ext(ckks_ctx* c, const uint64_t* host, int level, uint64_t* dev);

// ---- encoding (encode.cpp on the host, encode_gpu.hip on the device) ----
// host tables of the canonical-embedding encoder: root[k] = exp(-2 pi i k / N)
// (k < N/2) and twist[i] = exp(-i pi i / N) (i < N) as (re, im) pairs; pos[2j],
// pos[2j+1] = the FFT inputs of slot j and of its conjugate
void encode_tables(int N, std::vector<double>& root, std::vector<double>& twist, std::vector<uint32_t>& pos);
// count plaintexts of the slot values re (and im, may be null) [count][n], at
// `scale`, as residues over n_limbs limbs (modulus lm_mod(map, i)) in
// evaluation form: dev [count][n_limbs][N].  ESCALE if a coefficient leaves
// 63 bits.
void encode_gpu(ckks_ctx* c, const double* re, const double* im, size_t count, size_t n, double scale, int n_limbs,
                LimbMap map, uint64_t* dev);

// ---- sampling (sample.hip) ----
void sample_uniform(ckks_ctx* c, uint64_t* out, uint64_t seed, uint32_t kind, uint32_t a, uint32_t b0,
                    int n_limbs, LimbMap map, uint32_t b_step_per_limb);
void sample_small_rns(ckks_ctx* c, uint64_t* out, uint64_t seed, uint32_t kind, uint32_t a, uint32_t b,
                      int dist, int n_limbs, LimbMap map);   // dist 0 = ternary, 1 = CBD(21)
void keygen_swk(ckks_ctx* c, uint64_t seed, const uint64_t* s_ntt, const uint64_t* sp_ntt, uint64_t tag, uint64_t* key);
// ct = (-a s + e + m, a): e from the stream (5, ct_id) of seed, a from the
// stream (4, ct_id, prime) of a_seed, both in coefficient form, then NTT
void encrypt_sym(ckks_ctx* c, const uint64_t* s_ntt, const uint64_t* m_ntt, int level, uint64_t seed, uint64_t a_seed,
                 uint32_t ct_id, uint64_t* ct);
// the 'a' polynomials of `count` ciphertexts cts[count][2][level+1][N] (ct z
// from the stream (4, ct_id0 + z, prime) of a_seed), written in evaluation form;
// the first polynomials are not touched
void expand_seeded(ckks_ctx* c, uint64_t a_seed, uint32_t ct_id0, size_t count, int level, uint64_t* cts);
// residues below 2^bits (1 <= bits <= 64) to and from a bit stream of N * bits / 64 words per
// limb: count polynomials of n_limbs limbs, polynomial z at in + z * in_stride and
// out + z * out_stride (words); unpack = false packs
void pack_residues(ckks_ctx* c, const uint64_t* in, size_t in_stride, uint64_t* out, size_t out_stride,
                   int n_limbs, size_t count, int bits, bool unpack);
void ew_mul(ckks_ctx* c, uint64_t* out, const uint64_t* a, const uint64_t* b, int n_limbs, LimbMap map);
void decrypt_core(ckks_ctx* c, const uint64_t* ct, const uint64_t* s_ntt, int level, uint64_t* m);

}  // namespace ficgcn
