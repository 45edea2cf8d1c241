/*
 * ficgcn.h -- C ABI of the MI355X library for the encrypted GCN layer
 * X' = A_hat X W under RNS-CKKS (FicGCN, arXiv 2506.10399).
 *
 * Threat model (paper Sec. 2.4): the server holds A_hat and W in plaintext,
 * the client holds the secret key and sends X encrypted; the server computes
 * on ciphertexts and returns ciphertexts.  Calls marked [client] use the
 * secret key; [server] calls take only evaluation keys.
 *
 * Conventions shared by every entry point
 *  - Return value: ficgcn_status (0 = OK).  On failure nothing was enqueued
 *    unless the code is FICGCN_EDEVICE; ficgcn_last_error() gives a message
 *    (thread-local, valid until the next failing call on that thread).
 *  - Device buffers are caller-owned (e.g. torch tensors); the library never
 *    frees them.  Contexts, key sets and plans are library-owned handles,
 *    released with their *_destroy call.
 *  - Every device operation is enqueued on the context's HIP stream
 *    (ckks_ctx_set_stream; default: the null stream) and is asynchronous
 *    unless stated otherwise.  Host buffers passed to a call may be reused
 *    when the call returns.
 *  - Layout: a polynomial at level l is l+1 limbs of N uint64 words, limb i
 *    holding residues modulo q_i; a ciphertext is [2][l+1][N] (c0 limbs then
 *    c1 limbs), a plaintext [l+1][N].  Device ciphertexts and plaintexts are
 *    in the library's evaluation (NTT) representation; "coefficient form"
 *    host arrays hold the residues of the polynomial's coefficients.
 *  - Levels: q_0 > q_1 > ... > q_{L-1}; a rescale drops q_l.
 *  - Rotation by k maps slots (v_0..v_{M-1}) to (v_k..v_{M-1}, v_0..v_{k-1})
 *    (paper Sec. 2.1); negative k rotates right.
 */
#ifndef FICGCN_H
#define FICGCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FICGCN_OK = 0,
  FICGCN_EINVAL = -1,  /* bad argument (null pointer, size, unsupported parameter) */
  FICGCN_ELEVEL = -2,  /* level out of range or mismatched operands */
  FICGCN_ESCALE = -3,  /* scale or encoded value out of range */
  FICGCN_ENOKEY = -4,  /* a needed rotation / relinearisation key is missing */
  FICGCN_ENOMEM = -5,  /* device allocation failed */
  FICGCN_EDEVICE = -6, /* HIP runtime error */
  FICGCN_EPLAN = -7    /* plan cannot be built or does not match the call */
} ficgcn_status;

typedef struct ckks_ctx ckks_ctx;
typedef struct ckks_keys ckks_keys;
typedef struct ficgcn_plan ficgcn_plan;

/* CKKS parameters (paper Sec. 2.1; the sizes follow the workload table).
 * N = 2^log_n (2^9..2^17), M = N/2 slots; n_q primes of q_bits bits form Q,
 * n_p special primes of p_bits bits form P (hybrid key switching with
 * digits of n_p consecutive Q primes); scale = 2^log_scale. */
typedef struct {
  uint32_t log_n, n_q, q_bits, n_p, p_bits, log_scale;
} ckks_params;

const char* ficgcn_last_error(void);

/* ---------------------------------------------------------------- context */
/* RNS-CKKS context (paper Sec. 2.1; the paper takes its parameters from its
 * HE library, Sec. 4.1).  Builds the prime chain (the n_q largest primes
 * below 2^q_bits congruent to 1 mod 2N, descending, then the n_p largest
 * below 2^p_bits not already in Q), NTT tables and base-conversion constants
 * on the host; device tables follow on the first device call.  EINVAL for
 * log_n outside 9..17 or primes outside 20..61 bits.  *out is owned by the caller
 * (ckks_ctx_destroy).  Synchronous. */
ficgcn_status ckks_context_create(const ckks_params* p, ckks_ctx** out);
/* Releases a context (host and device tables); NULL is a no-op. */
void ckks_ctx_destroy(ckks_ctx* ctx);
/* Every later device call on ctx is enqueued on stream, a hipStream_t
 * (NULL = default stream); the caller keeps the stream alive. */
ficgcn_status ckks_ctx_set_stream(ckks_ctx* ctx, void* stream);
/* The RNS moduli of Sec. 2.1's ciphertext modulus: moduli_out[n_q + n_p],
 * Q primes (q_0 > q_1 > ...) then P primes.  Host only. */
ficgcn_status ckks_ctx_moduli(const ckks_ctx* ctx, uint64_t* moduli_out);
/* Galois element 5^(step mod M) mod 2N of the slot rotation Rot(., step)
 * of Sec. 2.1.  Host only. */
ficgcn_status ckks_galois_element(const ckks_ctx* ctx, int64_t step, uint64_t* g_out);
/* Waits for all work enqueued on the context's stream; EDEVICE carries the
 * first asynchronous HIP error. */
ficgcn_status ckks_sync(ckks_ctx* ctx);
/* Measurement infrastructure (no operation of the paper).
 * Kernel timing: while enabled, HIP events are recorded on the context's
 * stream around every launch of the instrumented kernels ("inter_fused":
 * the fused Inter-CA + combination pass, "comb_fused": the fused
 * combination of a SpIntra-CA layer,
 * "keymac", "moddown", "modup", "ntt").  profile_read synchronises the
 * stream, returns the summed event time and launch count of `kernel` since
 * the last read, and clears that kernel's record. */
ficgcn_status ficgcn_profile_enable(ckks_ctx* ctx, int on);
ficgcn_status ficgcn_profile_read(ckks_ctx* ctx, const char* kernel, double* ms_total, uint64_t* launches);

/* NTT autotuner (execution schedule of the Sec. 2.1 transform; no operation
 * of the paper): each limb's transform runs as a column pass of 2^s points
 * and a row pass of 2^(log_n - s) points (both between 2^4 and 2^9); times
 * every split s in {log_n/2 - 1, log_n/2, log_n/2 + 1} and workgroup width
 * pair (column pass x row pass) on 16 scratch polynomials of n_limbs limbs (a
 * key-switch batch's launch shape) with HIP events on the context's stream and
 * keeps the fastest for this context.  cols_out[3] receives (column width, row
 * width, s) (may be NULL).  Synchronous. */
ficgcn_status ckks_ntt_autotune(ckks_ctx* ctx, uint32_t n_limbs, int32_t* cols_out);
/* Sets the NTT schedule (as the autotuner would) directly: split s (0 = log_n / 2, else both passes
 * between 2^4 and 2^9 points) and the workgroup widths (1, 2, 4, 8 or 16).
 * Every schedule computes the same words.  EINVAL otherwise. */
ficgcn_status ckks_ntt_config(ckks_ctx* ctx, int32_t split, int32_t cols_column, int32_t cols_row);

/* ------------------------------------------------------------------ keys */
/* [client] Key generation of the threat model of Sec. 2.4 (the client owns
 * the secret; the server receives evaluation keys only) for the rotations
 * and products of Sec. 2.1.  Samples the ternary secret and the switching keys (rotation keys
 * for every step in rot_steps, the relinearisation key if with_relin) from
 * the ChaCha20 streams of `seed`.  *client_keys holds the secret and can
 * decrypt; *eval_keys holds only switching keys (what the server receives).
 * Either output pointer may be NULL if that object is not wanted. */
ficgcn_status ckks_keygen(ckks_ctx* ctx, uint64_t seed, const int64_t* rot_steps, size_t n_steps, int with_relin,
                          ckks_keys** client_keys, ckks_keys** eval_keys);
/* Number of switching keys held and their tags (Galois element; 0 = relin).
 * tags_out may be NULL (count only); up to cap tags written.  Host only. */
ficgcn_status ckks_keys_tags(const ckks_keys* keys, uint64_t* tags_out, size_t cap, size_t* n_out);
/* Copies one switching key (hybrid key switching, Sec. 2.1's rotation) to the
 * host in coefficient form, [beta][2][n_q + n_p][N] (b then a per digit);
 * host_out is caller-owned.  ENOKEY if the tag is absent.  Synchronous. */
ficgcn_status ckks_keys_export(ckks_ctx* ctx, const ckks_keys* keys, uint64_t tag, uint64_t* host_out);
/* Installs a switching key given in coefficient form (layout as export), for
 * a server that receives the client's evaluation keys (Sec. 2.4). */
ficgcn_status ckks_keys_import(ckks_ctx* ctx, ckks_keys* keys, uint64_t tag, const uint64_t* host_in);
/* An empty evaluation key set (Sec. 2.4's server side), to be filled with
 * ckks_keys_import; owned by the caller (ckks_keys_destroy). */
ficgcn_status ckks_keys_create_empty(ckks_ctx* ctx, ckks_keys** out);
/* Releases a key set (device keys, the secret of a client set); NULL is a no-op. */
void ckks_keys_destroy(ckks_keys* keys);

/* ------------------------------------------------- encode / encrypt [client] */
/* CKKS encoding of Sec. 2.1: n <= M complex slots (im may be NULL) at
 * `scale` into a caller-owned device plaintext [level+1][N]: round-half-even
 * of the scaled inverse canonical embedding (an FP64 FFT on the device), then
 * residues and NTT.  ESCALE if a scaled coefficient exceeds 63 bits. */
ficgcn_status ckks_encode(ckks_ctx* ctx, const double* re, const double* im, size_t n, double scale, uint32_t level,
                          uint64_t* pt_dev);
/* Batch form of the Sec. 2.1 encoding: `count` slot vectors of n doubles each
 * (real parts only, row-major, host memory), encoded on the device into
 * pt_dev[count][level+1][N]. */
ficgcn_status ckks_encode_batch(ckks_ctx* ctx, const double* re, size_t count, size_t n, double scale, uint32_t level,
                                uint64_t* pt_dev);
/* Uploads a plaintext (Sec. 2.1) given as coefficient-form residues
 * [level+1][N] (host) into a caller-owned device buffer, then NTT. */
ficgcn_status ckks_pt_load(ckks_ctx* ctx, const uint64_t* host_coeffs, uint32_t level, uint64_t* pt_dev);
/* [client] Symmetric CKKS encryption (Sec. 2.1; the client encrypts X,
 * Sec. 2.4): ct = (-a s + e + m, a) mod Q_level with a, e from the ChaCha20
 * streams of (seed, ct_id).  EINVAL without the secret. */
ficgcn_status ckks_encrypt(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* pt_dev, uint32_t level,
                           uint64_t seed, uint32_t ct_id, uint64_t* ct_dev);
/* [client] Symmetric CKKS encryption (Sec. 2.1) into a seeded ciphertext: as
 * ckks_encrypt, with e from the streams of (e_seed, ct_id) and the uniform part
 * a from those of a public seed, (a_seed, ct_id), so that the client may send
 * the first polynomial alone with (a_seed, ct_id) and the server rebuilds a with
 * ckks_expand_seeded.  The ciphertext words are ckks_encrypt's for e_seed with a
 * drawn from a_seed.  EINVAL without the secret, or if a_seed equals e_seed or
 * the key set's generation seed (a public seed must key no secret stream). */
ficgcn_status ckks_encrypt_seeded(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* pt_dev, uint32_t level,
                                  uint64_t e_seed, uint64_t a_seed, uint32_t ct_id, uint64_t* ct_dev);
/* [server] Rebuilds the uniform parts of `count` seeded ciphertexts (Sec. 2.1's
 * fresh encryption (-a s + e + m, a), a regenerated from its public seed):
 * cts_dev[count][2][level+1][N] (device, caller-owned), ciphertext z's second
 * polynomial is set to a of (a_seed, ct_id0 + z) in evaluation form, its first
 * polynomial (the client's c0) is not touched.  count = 0 is a no-op; ELEVEL
 * for a level outside the chain; EINVAL if the ids pass 2^32 - 1.  Asynchronous
 * on the context's stream. */
ficgcn_status ckks_expand_seeded(ckks_ctx* ctx, uint64_t a_seed, uint32_t ct_id0, size_t count, uint32_t level,
                                 uint64_t* cts_dev);
/* [either side] Transport form of residues (the RNS words of Sec. 2.1's
 * ciphertexts, no operation of the paper): n_limbs limbs of N residues below
 * 2^bits (in_dev, contiguous, device) become n_limbs * N * bits / 64 words
 * (out_dev, device, caller-owned): residue r of a limb holds bits r*bits ..
 * r*bits+bits-1 of the limb's little-endian bit stream; higher bits of a
 * residue are dropped.  With bits = the widest prime's bit length a
 * ciphertext's words shrink by that fraction of 64 (a 50-bit chain: 22%).
 * EINVAL for bits outside 1..64 or more than 65535 limbs; asynchronous on the
 * context's stream. */
ficgcn_status ckks_pack_residues(ckks_ctx* ctx, const uint64_t* in_dev, size_t n_limbs, uint32_t bits,
                                 uint64_t* out_dev);
/* [either side] The inverse of ckks_pack_residues: n_limbs packed limbs of
 * N * bits / 64 words (in_dev) to n_limbs limbs of N residues (out_dev). */
ficgcn_status ckks_unpack_residues(ckks_ctx* ctx, const uint64_t* in_dev, size_t n_limbs, uint32_t bits,
                                   uint64_t* out_dev);
/* [client] Decryption and decoding (Sec. 2.1, Sec. 2.4): n_slots slots
 * (im may be NULL) at `scale` into host arrays.  Synchronous. */
ficgcn_status ckks_decrypt(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* ct_dev, uint32_t level,
                           double scale, double* re, double* im, size_t n_slots);

/* -------------------------------------------------- transfers (either side) */
/* Uploads a ciphertext (Sec. 2.1) given in coefficient form
 * [2][level+1][N] (host) into a caller-owned device buffer, then NTT. */
ficgcn_status ckks_ct_load(ckks_ctx* ctx, const uint64_t* host_coeffs, uint32_t level, uint64_t* ct_dev);
/* Downloads a ciphertext (or, with n_polys = 1, a plaintext) of Sec. 2.1 in
 * coefficient form [n_polys][level+1][N] into caller-owned host memory.
 * Synchronous. */
ficgcn_status ckks_poly_store(ckks_ctx* ctx, const uint64_t* dev, uint32_t level, uint32_t n_polys,
                              uint64_t* host_coeffs);
/* The negacyclic number-theoretic transform under every RNS-CKKS product
 * (Sec. 2.1): forward (inverse = 0) or inverse, in place on n_limbs device
 * limbs starting at modulus index first_mod (Q primes 0..n_q-1, then P
 * primes); evaluation order is bit-reversed. */
ficgcn_status ckks_ntt(ckks_ctx* ctx, uint64_t* dev, uint32_t n_limbs, uint32_t first_mod, int inverse);

/* ------------------------------------------------------ evaluation [server] */
/* Rot of Sec. 2.1 (the dominant cost of SpIntra-CA, Sec. 3.3, and of the
 * App. A overhead table), hoisted.
 * Rotations of one ciphertext by each of steps[0..k): one ModUp of c1 is
 * shared by all k (hoisting).  Each rotation is computed as ModUp, then the
 * Galois automorphism on every extended digit, the key inner product and a
 * rounding ModDown (words equal to k single rotations).  outs[i] are k
 * device buffers [2][level+1][N]; a zero step copies the input.  ENOKEY if
 * a step's key is missing (nothing enqueued). */
ficgcn_status ckks_rotate_hoisted(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* ct_dev, uint32_t level,
                                  const int64_t* steps, size_t k, uint64_t* const* outs);
/* Rot of Sec. 2.1, batched over distinct ciphertexts.
 * n rotations Rot(cts[i], steps[i]) -> outs[i] at one level, run as one
 * key-switch batch (one ModUp per distinct input pointer, one inner-product
 * launch and one ModDown sequence for all n).  Words equal n single
 * rotations.  Outputs may not alias each other or any input; ENOKEY if a
 * step's key is missing (nothing enqueued). */
ficgcn_status ckks_rotate_batch(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* const* cts, uint32_t level,
                                const int64_t* steps, size_t n, uint64_t* const* outs);
/* PMult and Add of Sec. 2.1: acc += sum_i pts[i] (.) cts[i]
 * (plaintext-ciphertext multiply-accumulate of Sec. 3.3's masks and
 * Sec. 3.3.2's Inter-CA copies); every operand at `level`, caller-owned
 * device buffers; no rescale.  The *_op form below checks levels and scales. */
ficgcn_status ckks_pt_mul_acc(ckks_ctx* ctx, uint64_t* acc_dev, uint32_t level, const uint64_t* const* cts,
                              const uint64_t* const* pts, size_t k);
/* Constant multiplication of Sec. 2.1 for the combination X W (Sec. 3.2,
 * App. B): acc += sum_i consts[i] * cts[i] for signed integer constants (a
 * weight w encoded at scale s is round_half_even(w * s)); no rescale. */
ficgcn_status ckks_scalar_mul_acc(ckks_ctx* ctx, uint64_t* acc_dev, uint32_t level, const uint64_t* const* cts,
                                  const int64_t* consts, size_t k);
/* Add of Sec. 2.1: acc += in (ciphertexts at the same level). */
ficgcn_status ckks_add(ckks_ctx* ctx, uint64_t* acc_dev, const uint64_t* in_dev, uint32_t level);
/* Rescale of Sec. 2.1 (each multiplication consumes a level): in place,
 * round(c / q_level) on both components; the result is the ciphertext at
 * level-1, packed as [2][level][N] at the start of the buffer.  ELEVEL at
 * level 0. */
ficgcn_status ckks_rescale(ckks_ctx* ctx, uint64_t* ct_dev, uint32_t level);
/* CMult of Sec. 2.1 (the x^2 activation of Sec. 4.1's models): out = x * y
 * relinearised (tensor, then the relin key switches the a1 a2 term); no
 * rescale.  out may not alias x or y; ENOKEY without the relin key. */
ficgcn_status ckks_mul_relin(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* x_dev, const uint64_t* y_dev,
                             uint32_t level, uint64_t* out_dev);

/* ckks_mul_relin without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and the same output words as ckks_mul_relin;
 * its intermediates (tensor product, ModUp digits, inner products, ModDown
 * conversion: (3 (level+1) + ceil((level+1)/n_p) (level+1+n_p) + 2 (level+1+n_p))
 * limbs of N words) live in one fixed device array of
 * ckks_mul_relin_noalloc_limit() bytes (64 MiB) that each GPU holds from the
 * library's load until the process ends; a call that needs more returns
 * FICGCN_ENOMEM and enqueues nothing.  The context must already have its
 * device tables (any earlier device call on it, such as ckks_keygen, sets
 * them up; else EINVAL) and must belong to the current device.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller;
 * nothing in the array needs clearing between calls. */
ficgcn_status ckks_mul_relin_noalloc(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* x_dev,
                                     const uint64_t* y_dev, uint32_t level, uint64_t* out_dev);
size_t ckks_mul_relin_noalloc_limit(void);

/* ------------------------------------------- operands with level and scale
 * The same operations on descriptors that carry each operand's level and
 * scale (Sec. 2.1: a product's scale is the product of its factors' scales
 * and each multiplication consumes a level; a rescale divides the scale by
 * the prime it drops).  Every operand is checked before anything is
 * enqueued: ELEVEL when an operand sits at another level than the call
 * needs, ESCALE when a sum would add terms of different scales (relative
 * difference above 1e-9) or a scale is not positive, EINVAL for a null
 * buffer or a plaintext where a ciphertext is expected.  On success the
 * output descriptors' level and scale are updated; on failure nothing is
 * enqueued and no descriptor changes.  data stays caller-owned. */
typedef struct {
  uint64_t* data;    /* device buffer [n_poly][level+1][N], evaluation form */
  uint32_t level;
  uint32_t n_poly;   /* 2 = ciphertext, 1 = plaintext */
  double scale;
} ckks_operand;

/* [client] ckks_encrypt (Sec. 2.1, Sec. 2.4) of a plaintext operand into
 * ct->data; ct takes the plaintext's level and scale. */
ficgcn_status ckks_encrypt_op(ckks_ctx* ctx, const ckks_keys* client_keys, const ckks_operand* pt, uint64_t seed,
                              uint32_t ct_id, ckks_operand* ct);
/* [client] ckks_decrypt at the ciphertext's own level and scale. */
ficgcn_status ckks_decrypt_op(ckks_ctx* ctx, const ckks_keys* client_keys, const ckks_operand* ct, double* re,
                              double* im, size_t n_slots);
/* ckks_rotate_hoisted (Rot, Sec. 2.1): every outs[i] must be a ciphertext
 * buffer at in's level; each takes in's scale. */
ficgcn_status ckks_rotate_hoisted_op(ckks_ctx* ctx, const ckks_keys* eval_keys, const ckks_operand* in,
                                     const int64_t* steps, size_t k, ckks_operand* outs);
/* ckks_pt_mul_acc (PMult, Add, Sec. 2.1): cts and pts at acc's level; every
 * product's scale cts[i].scale * pts[i].scale must equal acc->scale, or,
 * when acc->scale is 0 (a fresh zero accumulator), the first product's. */
ficgcn_status ckks_pt_mul_acc_op(ckks_ctx* ctx, ckks_operand* acc, const ckks_operand* cts, const ckks_operand* pts,
                                 size_t k);
/* ckks_scalar_mul_acc (Sec. 3.2's combination): constants encoded at
 * const_scale; products' scales checked as in ckks_pt_mul_acc_op. */
ficgcn_status ckks_scalar_mul_acc_op(ckks_ctx* ctx, ckks_operand* acc, const ckks_operand* cts, const int64_t* consts,
                                     double const_scale, size_t k);
/* ckks_add (Sec. 2.1): equal levels and scales. */
ficgcn_status ckks_add_op(ckks_ctx* ctx, ckks_operand* acc, const ckks_operand* in);
/* ckks_rescale (Sec. 2.1): level -> level - 1, scale -> scale / q_level. */
ficgcn_status ckks_rescale_op(ckks_ctx* ctx, ckks_operand* ct);
/* ckks_mul_relin (CMult, Sec. 2.1): x, y and out at one level; out takes
 * x.scale * y.scale. */
ficgcn_status ckks_mul_relin_op(ckks_ctx* ctx, const ckks_keys* eval_keys, const ckks_operand* x,
                                const ckks_operand* y, ckks_operand* out);

/* ------------------------------------------------------------ plan [server] */
/* Plan options. */
typedef struct {
  int32_t first_mode;   /* 0: Inter-CA first layer (paper's rule), 1: SpIntra-CA (one-layer models only) */
  int32_t use_noo;      /* node order optimisation (Alg. 1) on/off */
  int32_t family;       /* SpIntra-CA routing: 0 = cheaper of 1 and 2, 1 = diagonal, 2 = baby-step/giant-step,
                           3 = the paper's radix-2 routing with per-round masks (Sec. 3.3): one level per
                           round in which something moves, so the chain needs that many spare primes;
                           4 = diagonal with double hoisting: every rotation's key inner product is multiplied
                           by its mask on the key basis (Q_l and P) and summed before one ModDown per output;
                           its masks carry level + 1 + alpha limbs */
  int32_t TH;           /* region size cap; 0 = 1024 below 10000 nodes, else 4096 */
  int32_t activation;   /* x^2 after every layer */
  int32_t t;            /* SpIntra-CA packing: columns per ciphertext, a power of two no larger than
                           next_pow2(F') and M / next_pow2(n_v); 0 = the paper's rule (Sec. 3.2, App. B) */
  int32_t aoo_off;      /* family 3 with t = 1: route each shift pi(u) - pi(v) as it is instead of the
                           shorter way round the ring (AOO, Sec. 3.3.1, off: for its ablation) */
  double cpoo;          /* family 3: CPOO sparsity threshold in [0, 1] (Sec. 3.3.1; the paper's ablation,
                           Sec. 4.2.2, finds 0.2-0.3 best); 0 = CPOO off */
  int32_t first_pack;   /* Inter-CA first layer's packing (Sec. 3.2, App. B): 0 = one input column per
                           ciphertext (combination as integer-weight sums); -1 = the paper's rule: when
                           M > N F', the case-1 layout at the argmin t of J(t; F, n) = 2 ceil(F n / t)
                           + 20 ceil(log2 t) over powers of two with t pow2(F') pow2(N) <= M (halved
                           while a later layer is wider than t pow2(F')), else 0; t > 0 = the case-1
                           layout at that t.  In the case-1 layout ciphertext j of copy k holds input
                           columns j t .. j t + t - 1, each repeated for the F' output columns in
                           blocks of Bc = M / (t pow2(F')) slots, node v at offset pi(v); the layer's
                           operands are A_hat_k (x) W-slices, its ceil(log2 t) rotations fold the
                           column blocks, and it outputs one ciphertext whose block l holds output
                           column l; later layers combine such blocks by block rotations */
  double agg_c;         /* the factor c of Sec. 3.3.2's aggregation-mode formula (0 = 1.0) */
  int32_t low_level;    /* 1: the first layer's inputs sit at the lowest level the layers need (their
                           rescales, Sec. 2.1, plus one spare prime for the output) instead of the top
                           of the chain; the client encrypts at plan info level_in of layer 0 */
  double max_key_bytes; /* plan search only: a candidate whose rotation keys take more device memory
                           than this is infeasible (0 = no limit) */
} ficgcn_plan_opts;

/* The server's plan of the method (Sec. 3.1's workflow): latency-aware
 * packing (Sec. 3.2, App. B), aggregation mode per layer (Sec. 3.3.2, App.
 * B), SpIntra-CA shift routing (Sec. 3.3, 3.3.1) and node order (Sec. 3.4,
 * Alg. 1) for the GCN of Sec. 2.2.
 * Builds the plan of an n_layers-layer GCN over the normalised adjacency
 * A_hat given as CSR (row v: columns col[rowptr[v]..rowptr[v+1]) with values
 * val, the diagonal included): node order, per-layer aggregation mode,
 * packing, shift routing, scale schedule and integer weights.  weights[l]
 * is the dims[l] x dims[l+1] row-major FP64 matrix of layer l.  The
 * plaintext operands (Inter-CA copies' adjacency plaintexts, masks) are
 * encoded by ficgcn_plan_encode or loaded with ficgcn_plan_load_operand. */
ficgcn_status ficgcn_plan_create(ckks_ctx* ctx, const int32_t* rowptr, const int32_t* col, const double* val,
                                 uint32_t n_v, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                                 const ficgcn_plan_opts* opts, ficgcn_plan** out);
/* Releases a plan with its operands and graphs; NULL is a no-op. */
void ficgcn_plan_destroy(ficgcn_plan* plan);
/* The node order of Sec. 3.4 / Alg. 1: pi_out[v] (n_v int32, host) = slot of
 * node v inside a column block (the client packs its inputs in this order,
 * App. B's node order back propagation). */
ficgcn_status ficgcn_plan_node_order(const ficgcn_plan* plan, int32_t* pi_out);
/* Inter-CA copy structure of layer `layer` (the client builds its encrypted
 * copies from it, paper Sec. 3.3.2): src_out[k * n_v + v] = the node whose
 * features copy k holds at node v's slot, -1 for none; copy 0 is the node
 * itself.  K = info "K". */
ficgcn_status ficgcn_plan_copy_sources(const ficgcn_plan* plan, uint32_t layer, int32_t* src_out);
/* Rotation steps of the plan's Rot operations (Sec. 3.3's SpIntra-CA shifts,
 * Sec. 3.2's packing folds), whose keys the client must generate (Sec. 2.4):
 * sorted, in [1, M); steps_out may be NULL (count only). */
ficgcn_status ficgcn_plan_rot_steps(const ficgcn_plan* plan, int64_t* steps_out, size_t cap, size_t* n_out);
/* Plan description: per layer {kind, f_in, f_out, K, t, B, family, G,
 * n_shifts, level_in, level_out, n_in_cts, n_out_cts, pack (1 = the case-1
 * layout of an Inter-CA layer), comb (1 = block-rotation combination of a
 * packed input), fold rotations, combination offsets, paper_mode (Sec. 3.3.2's
 * formula for a later layer: 0 Inter-CA, 1 SpIntra-CA, -1 not evaluated)} as
 * int64, 18 per layer, then 5 doubles per layer in scales_out {scale_in,
 * scale_out, weight scale, Inter-CA cost 2 ceil(F n / t), SpIntra-CA cost
 * 10 c n log2(N)^2}.  The executed mode of a later layer is SpIntra-CA either
 * way: an Inter-CA later layer would first build its K neighbour copies from
 * the previous layer's ciphertext by rotations and masks, and those copies'
 * products with the K adjacency plaintexts merge into exactly the diagonal
 * SpIntra-CA form. */
ficgcn_status ficgcn_plan_info(const ficgcn_plan* plan, int64_t* info_out, double* scales_out, uint32_t* n_layers);
/* Shifts pi(u) - pi(v) routed by layer `layer`'s SpIntra-CA aggregation
 * (Sec. 3.3, shortest way round the ring per Sec. 3.3.1's AOO), sorted. */
ficgcn_status ficgcn_plan_shifts(const ficgcn_plan* plan, uint32_t layer, int64_t* out, size_t cap, size_t* n_out);
/* Integer weights of a layer's combination (Sec. 3.2's X W) as the plan
 * encodes them: round_half_even(w * sW), dims[l] x dims[l+1] int64. */
ficgcn_status ficgcn_plan_weights_int(const ficgcn_plan* plan, uint32_t layer, int64_t* out);
/* The plaintext operands of a layer: Sec. 3.3's masks or Sec. 3.3.2's
 * Inter-CA adjacency plaintexts.
 * Number of plaintext operands of a layer and the slot vector of operand i
 * (M doubles): Inter-CA adjacency plaintext of copy i, or SpIntra-CA mask i
 * (families 1 and 2: packed ciphertext i / n_shifts, shift index
 * i % n_shifts; family 3: see ficgcn_plan_radix2_stats). */
ficgcn_status ficgcn_plan_operand_count(const ficgcn_plan* plan, uint32_t layer, size_t* n_out);
ficgcn_status ficgcn_plan_operand_slots(const ficgcn_plan* plan, uint32_t layer, size_t i, double* slots_out);
/* Level and encoding scale of operand i (the Inter-CA plaintexts sit at the
 * layer's input level, the masks of families 1, 2 and 4 at the aggregation
 * level; a radix-2 mask sits at the level of the step that multiplies it and
 * is encoded at that level's prime, which the step's rescale drops).  Family
 * 4 masks hold level + 1 + alpha limbs: the Q_0..Q_level residues, then the
 * special primes' (ficgcn_plan_load_operand takes them in that order). */
ficgcn_status ficgcn_plan_operand_level(const ficgcn_plan* plan, uint32_t layer, size_t i, uint32_t* level_out,
                                        double* scale_out);
/* Radix-2 aggregation program of a family-3 layer (Sec. 3.3 with CPOO of
 * Sec. 3.3.1), 8 int64: {working ciphertexts created by the first-fit
 * assignment, steps, distinct (ciphertext, amount) rotations, distinct
 * rotation amounts, levels consumed, masks per packed ciphertext, demands
 * moved by CPOO merging, intermediate ciphertexts}.  Operand i of the layer
 * is mask i % (masks per packed ciphertext) of packed ciphertext
 * i / (masks per packed ciphertext).  EPLAN for other layers. */
ficgcn_status ficgcn_plan_radix2_stats(const ficgcn_plan* plan, uint32_t layer, int64_t* out);
/* Encodes every operand (Sec. 2.1's encoding of the masks and adjacency
 * plaintexts) with the library's device encoder.  Synchronous. */
ficgcn_status ficgcn_plan_encode(ckks_ctx* ctx, ficgcn_plan* plan);
/* Installs operand i of a layer (Sec. 3.3's masks, Sec. 3.3.2's plaintexts)
 * from coefficient-form host residues [level+1][N] at the operand's level
 * (ficgcn_plan_operand_level), for operands encoded elsewhere.  EINVAL for an
 * index out of range. */
ficgcn_status ficgcn_plan_load_operand(ckks_ctx* ctx, ficgcn_plan* plan, uint32_t layer, size_t i,
                                       const uint64_t* host_coeffs);

/* Measurement only (no operation of the paper).
 * Fills every operand of the plan with uniform residues drawn on the device
 * (ChaCha20 stream (6, layer * 2^20 + operand, limb) of `seed`, one the
 * scheme never uses).  For latency measurement only: the layer runs exactly
 * as with encoded operands, but its words mean nothing. */
ficgcn_status ficgcn_plan_fill_operands(ckks_ctx* ctx, ficgcn_plan* plan, uint64_t seed);

/* One encrypted GCN layer X' = A_hat X W (Sec. 2.2, the problem statement of
 * Sec. 3): Inter-CA (Sec. 3.3.2) or SpIntra-CA (Sec. 3.3) aggregation, the
 * combination and packing of Sec. 3.2 / App. B, rescales (Sec. 2.1) and the
 * x^2 activation, as the plan schedules them.  Server side (Sec. 2.4):
 * evaluation keys only; ENOKEY if a key is missing, EPLAN if the buffers do
 * not match the plan (counts, levels), nothing enqueued then.
 * Inputs: Inter-CA first layer: K*F client ciphertexts, copy k of column f at
 * index k*F + f; later / SpIntra-CA layers: the previous layer's outputs.
 * mode 0 = one library operation at a time ("plain"), mode 1 = fused,
 * batched launches ("batched"), mode 2 = the batched launch sequence
 * captured in a HIP graph: the first call for a given set of input and
 * output buffers and keys runs mode 1 while recording its device tables,
 * then captures; later calls with the same buffers replay the graph (the
 * plan keeps one graph per layer; new buffers recapture).  All three
 * produce the same words.  With in_cts NULL and n_in 0 an Inter-CA layer
 * reads the inputs ficgcn_plan_pack_inputs rearranged for it (modes 1 and 2;
 * the same words as from the ciphertexts themselves); EPLAN otherwise. */
ficgcn_status ficgcn_gcn_layer(ckks_ctx* ctx, const ckks_keys* eval_keys, const ficgcn_plan* plan, uint32_t layer,
                               const uint64_t* const* in_cts, size_t n_in, uint64_t* const* out_cts, size_t n_out,
                               int32_t mode);

/* Inputs of an Inter-CA layer stored as the operands of its matrix-core pass
 * (Sec. 3.3.2's aggregation fused with App. B's combination): for each wave
 * of the pass (16 coefficients of one limb of one component) and each (copy,
 * 64-feature block), the seven balanced base-256 digit planes of its 64 lanes:
 * digits 0..5 as int8 planes of 16 bytes per lane, digit 6 (in [0, 8] for a
 * residue below 2^51) as 4-bit values, 8 bytes per lane.  6.5 bytes per
 * residue instead of 8, and no digit work in the pass.  packed_input_words:
 * the buffer size in 64-bit words (K copies x ceil(F / 64) blocks x (N / 16)
 * x (level + 1) x 2 waves x 832 words); EPLAN if the layer is not Inter-CA or
 * a prime of the chain is 2^51 or more. */
ficgcn_status ficgcn_plan_packed_input_words(const ficgcn_plan* plan, ckks_ctx* ctx, uint32_t layer,
                                             uint64_t* words_out);
/* Rearranges the layer's K*F input ciphertexts (as for ficgcn_gcn_layer)
 * into packed_dev (caller-owned device buffer of at least packed_words
 * words; it must stay allocated while the plan may read it) and registers it
 * with the plan's layer.  Synchronous.  EPLAN if the layer is not Inter-CA or
 * its shape or weights are outside the matrix-core pass (K <= 16, F <= 16384,
 * integer weights within 7 balanced digits); EINVAL if a prime of the chain
 * is 2^51 or more or the buffer is too small. */
ficgcn_status ficgcn_plan_pack_inputs(ckks_ctx* ctx, ficgcn_plan* plan, uint32_t layer, const uint64_t* const* in_cts,
                                      size_t n_in, uint64_t* packed_dev, uint64_t packed_words);

/* ------------------------------------------------------ plan search [server]
 * The packing and node-order choice as a search over candidate plans
 * (packing t of Sec. 3.2, NOO on/off and its region cap TH of Sec. 3.4, the
 * SpIntra-CA routing family).  The analytic judge scores a built plan by the
 * algorithmic HBM bytes of its batched execution; a learned cost model
 * (below) may prune the candidates before any plan is built. */

/* Number of floats ficgcn_candidate_features writes. */
#define FICGCN_N_FEATURES 24

/* Candidates of Sec. 3.2's packing (t), Sec. 3.4's NOO (on/off, TH) and the
 * routing family.
 * Enumerates the candidate options for this graph size and model: every
 * feasible t, NOO off (when the graph fits one column block) or on with TH
 * in {64, 256, 1024, 4096} below n_v (plus TH = n_v), families 1, 2 and 4;
 * the other fields are copied from base.  Writes up to cap entries, *n_out =
 * the full count.  Host only. */
ficgcn_status ficgcn_plan_candidates(uint32_t n_v, const uint32_t* dims, uint32_t n_layers, uint32_t log_n,
                                     const ficgcn_plan_opts* base, ficgcn_plan_opts* out, size_t cap,
                                     size_t* n_out);
/* Features for the learned cost model (the paper quantifies such effects by
 * its factor c, Sec. 3.3.2, and notes that conflicts resist a closed form,
 * App. C).
 * Local-adjacency features of one candidate, computed from the CSR graph
 * (as ficgcn_plan_create takes it) without building the plan: degree
 * statistics, locality of the given node order, shift counts of the
 * identity order, and the candidate's t, B, TH, family.  Host only; out
 * holds FICGCN_N_FEATURES floats. */
ficgcn_status ficgcn_candidate_features(const int32_t* rowptr, const int32_t* col, uint32_t n_v, const uint32_t* dims,
                                        uint32_t n_layers, uint32_t log_n, const ficgcn_plan_opts* opts, float* out);
/* Analytic judge in the role of App. B's latency-aware objective, in bytes:
 * algorithmic HBM bytes of one batched inference of the
 * plan (inputs, keys, masks and outputs of every operation, per the key
 * switching, MAC and rescale byte counts), as a double.  Host only. */
ficgcn_status ficgcn_plan_cost(const ficgcn_plan* plan, double* bytes_out);

typedef struct ficgcn_mlp ficgcn_mlp;

typedef struct {
  uint32_t n_candidates;   /* candidates enumerated */
  uint32_t n_built;        /* plans built and judged */
  double best_cost;        /* judge's bytes of the chosen plan */
  double build_seconds;    /* host time spent building candidate plans */
} ficgcn_search_stats;

/* The packing / node-order search of Sec. 3.2 and Sec. 3.4 (App. B's
 * objective as the judge).  Picks the options of the plan to build.  model == NULL: exhaustive
 * analytic search (every candidate built and judged).  Otherwise the model
 * predicts each candidate's latency from its features, the `keep` fastest
 * predictions are built and judged, and the judge's best of those wins
 * (every candidate is the fallback when none of the kept builds).  The
 * model runs on the context's device. */
ficgcn_status ficgcn_plan_search(ckks_ctx* ctx, const int32_t* rowptr, const int32_t* col, const double* val,
                                 uint32_t n_v, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                                 const ficgcn_plan_opts* base, ficgcn_mlp* model, uint32_t keep,
                                 ficgcn_plan_opts* best_out, ficgcn_search_stats* stats_out);

/* ------------------------------------------------ learned cost model [server]
 * A fully connected network widths[0] -> ... -> widths[n-1] with ReLU after
 * every layer but the last, fp32, trained by mean squared error with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Parameters are packed layer by layer
 * as W_j [widths[j+1]][widths[j]] then b_j [widths[j+1]]; the caller
 * supplies the initial values (host).  Forward, backward and Adam run in the
 * library's kernels on the context's stream; x and y are device buffers
 * [n][widths[0]] and [n][widths[n-1]]. */
ficgcn_status ficgcn_mlp_create(ckks_ctx* ctx, const uint32_t* widths, uint32_t n_widths, const float* params,
                                ficgcn_mlp** out);
void ficgcn_mlp_destroy(ficgcn_mlp* mlp);
ficgcn_status ficgcn_mlp_param_count(const ficgcn_mlp* mlp, size_t* n_out);
/* Copies the parameters to host memory (n_params floats). */
ficgcn_status ficgcn_mlp_get_params(const ficgcn_mlp* mlp, float* params_out);
/* y = network(x) for n rows. */
ficgcn_status ficgcn_mlp_forward(ficgcn_mlp* mlp, const float* x_dev, uint32_t n, float* y_dev);
/* Loss mean((network(x) - y)^2) and its gradient (n_params floats), both to
 * host memory; parameters unchanged. */
ficgcn_status ficgcn_mlp_gradient(ficgcn_mlp* mlp, const float* x_dev, const float* y_dev, uint32_t n,
                                  float* loss_out, float* grad_out);
/* One Adam step on the batch (x, y) with learning rate lr; *loss_out gets the
 * batch loss before the step. */
ficgcn_status ficgcn_mlp_train_step(ficgcn_mlp* mlp, const float* x_dev, const float* y_dev, uint32_t n, float lr,
                                    float* loss_out);

/* ----------------------------------------------------------- serving [server]
 * Continuous batching of encrypted GCN inferences (the method's layer,
 * Sec. 3, served to many clients under the threat model of Sec. 2.4) on one
 * GPU.  The server runs up to n_slots requests at once, each on its own
 * context and stream (so their kernels overlap on the device), admits waiting
 * requests in FIFO order as slots and device memory free up (a later request
 * that fits may pass the head until the head has been passed 16 times), and
 * keeps every client's evaluation keys resident (the caller's ckks_keys
 * objects, which must outlive the server).
 * Device memory is accounted in full against hbm_budget_bytes: the resident
 * key sets (each distinct set from its first request on), per distinct plan
 * its operands and weight tables (server-side data, encoded once), and per
 * slot an arena and a scratch share.  A request's arena holds its input
 * ciphertexts and every layer's outputs; its scratch share is bounded from the
 * plan (key-switch chunk buffers, rotated ciphertexts and inner sums, the
 * encoder's chunk, 64 ciphertexts).  Arenas only grow, so in steady state a
 * request allocates nothing; idle slots' arenas and scratch are released when
 * a waiting request needs the room.  The first request of a plan encodes its
 * operands (or loads the request's operands_host) and builds its tables; any
 * number of requests may then run one plan at once. */
typedef struct ficgcn_server ficgcn_server;

typedef struct {
  const ficgcn_plan* plan;         /* the graph's plan (server side); must outlive the server */
  const ckks_keys* eval_keys;      /* the client's keys, resident on the device */
  const uint64_t* inputs_host;     /* n_in client ciphertexts [n_in][2][level_in+1][N] in host memory
                                      (pinned for an asynchronous upload; evaluation-form words as the
                                      device holds them); read while the request runs; see `seeded` */
  size_t n_in;
  uint64_t* output_host;           /* the last layer's n_out ciphertexts [n_out][2][level_out+1][N] */
  size_t n_out;
  const uint64_t* const* operands_host;  /* taken from the plan's first submitted request only (kept
                                      alive until that request is waited for): NULL = the plan's operands
                                      are encoded on the device (ficgcn_plan_encode); else per layer,
                                      every operand's coefficient-form residues in operand order, as
                                      ficgcn_plan_load_operand takes them, concatenated */
  uint32_t seeded;                 /* nonzero: the inputs are seeded ciphertexts (ckks_encrypt_seeded) and
                                      inputs_host holds each one's first polynomial only,
                                      [n_in][level_in+1][N]; input i's second polynomial is rebuilt on the
                                      device from (a_seed, a_id0 + i), as ckks_expand_seeded does */
  uint32_t a_id0;
  uint64_t a_seed;
  uint32_t packed_bits;            /* seeded inputs only: 0 = first polynomials as words; else each input's
                                      first polynomial packed at packed_bits per residue
                                      (ckks_pack_residues), [n_in][(level_in+1) N packed_bits / 64] words;
                                      at least the bit length of every prime at level_in (else EINVAL) */
} ficgcn_request;

typedef struct {
  int32_t status;                  /* the request's ficgcn_status */
  double queue_ms, run_ms, latency_ms;   /* submission to admission, admission to completion, total */
  uint64_t footprint_bytes;        /* arena bytes plus the scratch bound */
} ficgcn_request_result;

typedef struct {
  uint32_t completed, failed;
  double p50_ms, p99_ms, mean_ms;  /* latency (submission to completion), nearest-rank percentiles */
  double throughput_per_s;         /* completed requests / (last completion - first submission) */
  uint64_t peak_bytes;             /* largest device memory held: resident keys and tables, arenas, scratch */
  uint32_t max_concurrent;         /* most requests running at once */
  uint64_t resident_bytes;         /* key sets and plan tables */
  uint64_t arena_allocs;           /* arena (re)allocations over the server's life */
  uint64_t scratch_overruns;       /* requests whose measured scratch exceeded the bound (then counted) */
} ficgcn_server_summary;

/* Creates the slots (contexts for params on the current device, one stream
 * each, at the default priority) and their worker threads. */
ficgcn_status ficgcn_server_create(const ckks_params* params, uint32_t n_slots, uint64_t hbm_budget_bytes,
                                   ficgcn_server** out);
/* Stops the workers after their running requests; waiting requests are dropped. */
void ficgcn_server_destroy(ficgcn_server* server);
/* Queues a request; ENOMEM if it can never fit the budget (with the resident
 * keys and plans), EINVAL if its plan or keys have other parameters. */
ficgcn_status ficgcn_server_submit(ficgcn_server* server, const ficgcn_request* req, uint64_t* id_out);
/* Blocks until the request completes; returns its status. */
ficgcn_status ficgcn_server_wait(ficgcn_server* server, uint64_t id, ficgcn_request_result* out);
ficgcn_status ficgcn_server_stats(ficgcn_server* server, ficgcn_server_summary* out);

#ifdef __cplusplus
}
#endif
#endif
