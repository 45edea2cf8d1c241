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
/* Builds the prime chain (the n_q largest primes below 2^q_bits congruent to
 * 1 mod 2N, descending, then the n_p largest below 2^p_bits), NTT tables
 * and base-conversion constants on the current HIP device.  Synchronous. */
ficgcn_status ckks_context_create(const ckks_params* p, ckks_ctx** out);
void ckks_ctx_destroy(ckks_ctx* ctx);
/* stream: a hipStream_t (NULL = default stream). */
ficgcn_status ckks_ctx_set_stream(ckks_ctx* ctx, void* stream);
/* moduli_out[n_q + n_p]: Q primes then P primes. */
ficgcn_status ckks_ctx_moduli(const ckks_ctx* ctx, uint64_t* moduli_out);
/* Galois element 5^(step mod M) mod 2N of a slot rotation. */
ficgcn_status ckks_galois_element(const ckks_ctx* ctx, int64_t step, uint64_t* g_out);
/* Waits for all work enqueued on the context's stream. */
ficgcn_status ckks_sync(ckks_ctx* ctx);
/* Kernel timing: while enabled, HIP events are recorded on the context's
 * stream around every launch of the instrumented kernels ("inter_fused":
 * the fused Inter-CA + combination pass, "comb_fused": the fused
 * combination of a SpIntra-CA layer,
 * "keymac", "moddown", "modup", "ntt").  profile_read synchronises the
 * stream, returns the summed event time and launch count of `kernel` since
 * the last read, and clears that kernel's record. */
ficgcn_status ficgcn_profile_enable(ckks_ctx* ctx, int on);
ficgcn_status ficgcn_profile_read(ckks_ctx* ctx, const char* kernel, double* ms_total, uint64_t* launches);

/* NTT autotuner: each limb's transform runs as a column pass of 2^s points
 * and a row pass of 2^(log_n - s) points (both between 2^4 and 2^9); times
 * every split s in {log_n/2 - 1, log_n/2, log_n/2 + 1} and workgroup width
 * pair (column pass x row pass) on 16 scratch polynomials of n_limbs limbs (a
 * key-switch batch's launch shape) with HIP events on the context's stream and
 * keeps the fastest for this context.  cols_out[3] receives (column width, row
 * width, s) (may be NULL).  Synchronous. */
ficgcn_status ckks_ntt_autotune(ckks_ctx* ctx, uint32_t n_limbs, int32_t* cols_out);
/* Sets the NTT schedule directly: split s (0 = log_n / 2, else both passes
 * between 2^4 and 2^9 points) and the workgroup widths (1, 2, 4, 8 or 16).
 * Every schedule computes the same words.  EINVAL otherwise. */
ficgcn_status ckks_ntt_config(ckks_ctx* ctx, int32_t split, int32_t cols_column, int32_t cols_row);

/* ------------------------------------------------------------------ keys */
/* [client] Samples the ternary secret and the switching keys (rotation keys
 * for every step in rot_steps, the relinearisation key if with_relin) from
 * the ChaCha20 streams of `seed`.  *client_keys holds the secret and can
 * decrypt; *eval_keys holds only switching keys (what the server receives).
 * Either output pointer may be NULL if that object is not wanted. */
ficgcn_status ckks_keygen(ckks_ctx* ctx, uint64_t seed, const int64_t* rot_steps, size_t n_steps, int with_relin,
                          ckks_keys** client_keys, ckks_keys** eval_keys);
/* Number of switching keys held and their tags (Galois element; 0 = relin). */
ficgcn_status ckks_keys_tags(const ckks_keys* keys, uint64_t* tags_out, size_t cap, size_t* n_out);
/* Copies one switching key to the host in coefficient form,
 * [beta][2][n_q + n_p][N] (b then a per digit).  Synchronous. */
ficgcn_status ckks_keys_export(ckks_ctx* ctx, const ckks_keys* keys, uint64_t tag, uint64_t* host_out);
/* Installs a switching key given in coefficient form (layout as export). */
ficgcn_status ckks_keys_import(ckks_ctx* ctx, ckks_keys* keys, uint64_t tag, const uint64_t* host_in);
/* An empty evaluation key set, to be filled with ckks_keys_import. */
ficgcn_status ckks_keys_create_empty(ckks_ctx* ctx, ckks_keys** out);
void ckks_keys_destroy(ckks_keys* keys);

/* ------------------------------------------------- encode / encrypt [client] */
/* Encodes n <= M complex slots (im may be NULL) at `scale` into a device
 * plaintext [level+1][N]: round-half-even of the scaled inverse canonical
 * embedding (FP64 FFT on the host), then residues and NTT. */
ficgcn_status ckks_encode(ckks_ctx* ctx, const double* re, const double* im, size_t n, double scale, uint32_t level,
                          uint64_t* pt_dev);
/* Batch form: `count` slot vectors of n doubles each (real parts only,
 * row-major), encoded on host threads into pt_dev[count][level+1][N]. */
ficgcn_status ckks_encode_batch(ckks_ctx* ctx, const double* re, size_t count, size_t n, double scale, uint32_t level,
                                uint64_t* pt_dev);
/* Uploads a plaintext given as coefficient-form residues [level+1][N]. */
ficgcn_status ckks_pt_load(ckks_ctx* ctx, const uint64_t* host_coeffs, uint32_t level, uint64_t* pt_dev);
/* ct = (-a s + e + m, a) mod Q_level with a, e from the streams of (seed, ct_id). */
ficgcn_status ckks_encrypt(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* pt_dev, uint32_t level,
                           uint64_t seed, uint32_t ct_id, uint64_t* ct_dev);
/* Decrypts and decodes n_slots slots (im may be NULL) at `scale`.  Synchronous. */
ficgcn_status ckks_decrypt(ckks_ctx* ctx, const ckks_keys* client_keys, const uint64_t* ct_dev, uint32_t level,
                           double scale, double* re, double* im, size_t n_slots);

/* -------------------------------------------------- transfers (either side) */
/* Uploads a ciphertext given in coefficient form [2][level+1][N]. */
ficgcn_status ckks_ct_load(ckks_ctx* ctx, const uint64_t* host_coeffs, uint32_t level, uint64_t* ct_dev);
/* Downloads a ciphertext (or, with n_polys = 1, a plaintext) in coefficient
 * form [n_polys][level+1][N].  Synchronous. */
ficgcn_status ckks_poly_store(ckks_ctx* ctx, const uint64_t* dev, uint32_t level, uint32_t n_polys,
                              uint64_t* host_coeffs);
/* Forward (inverse = 0) or inverse NTT in place on n_limbs limbs starting at
 * modulus index first_mod (Q primes 0..n_q-1, then P primes). */
ficgcn_status ckks_ntt(ckks_ctx* ctx, uint64_t* dev, uint32_t n_limbs, uint32_t first_mod, int inverse);

/* ------------------------------------------------------ evaluation [server] */
/* Rotations of one ciphertext by each of steps[0..k): one ModUp of c1 is
 * shared by all k (hoisting).  Each rotation is computed as ModUp, then the
 * Galois automorphism on every extended digit, the key inner product and a
 * rounding ModDown (words equal to k single rotations).  outs[i] are k
 * device buffers [2][level+1][N]; a zero step copies the input.  ENOKEY if
 * a step's key is missing (nothing enqueued). */
ficgcn_status ckks_rotate_hoisted(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* ct_dev, uint32_t level,
                                  const int64_t* steps, size_t k, uint64_t* const* outs);
/* n rotations Rot(cts[i], steps[i]) -> outs[i] at one level, run as one
 * key-switch batch (one ModUp per distinct input pointer, one inner-product
 * launch and one ModDown sequence for all n).  Words equal n single
 * rotations.  Outputs may not alias each other or any input; ENOKEY if a
 * step's key is missing (nothing enqueued). */
ficgcn_status ckks_rotate_batch(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* const* cts, uint32_t level,
                                const int64_t* steps, size_t n, uint64_t* const* outs);
/* acc += sum_i pts[i] (.) cts[i]  (plaintext-ciphertext multiply-accumulate
 * of Sec. 3.3's masks and Inter-CA copies); no rescale. */
ficgcn_status ckks_pt_mul_acc(ckks_ctx* ctx, uint64_t* acc_dev, uint32_t level, const uint64_t* const* cts,
                              const uint64_t* const* pts, size_t k);
/* acc += sum_i consts[i] * cts[i] for signed integer constants (a weight w
 * encoded at scale s is round_half_even(w * s)); no rescale. */
ficgcn_status ckks_scalar_mul_acc(ckks_ctx* ctx, uint64_t* acc_dev, uint32_t level, const uint64_t* const* cts,
                                  const int64_t* consts, size_t k);
/* acc += in (ciphertexts at the same level). */
ficgcn_status ckks_add(ckks_ctx* ctx, uint64_t* acc_dev, const uint64_t* in_dev, uint32_t level);
/* In place: round(c / q_level) on both components; the result is the
 * ciphertext at level-1, packed as [2][level][N] at the start of the buffer. */
ficgcn_status ckks_rescale(ckks_ctx* ctx, uint64_t* ct_dev, uint32_t level);
/* out = x * y relinearised (tensor, then the relin key switches the a1 a2
 * term); no rescale.  out may not alias x or y. */
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
} ficgcn_plan_opts;

/* Builds the plan of an n_layers-layer GCN over the normalised adjacency
 * A_hat given as CSR (row v: columns col[rowptr[v]..rowptr[v+1]) with values
 * val, the diagonal included): node order, per-layer aggregation mode,
 * packing, shift routing, scale schedule and integer weights.  weights[l]
 * is the dims[l] x dims[l+1] row-major FP64 matrix of layer l.  The
 * plaintext operands (Inter-CA copies' adjacency plaintexts, masks) are
 * encoded by ficgcn_plan_encode or loaded with ficgcn_plan_load_operand. */
ficgcn_status ficgcn_plan_create(ckks_ctx* ctx, const int32_t* rowptr, const int32_t* col, const double* val,
                                 uint32_t n_v, const uint32_t* dims, uint32_t n_layers, const double* const* weights,
                                 const ficgcn_plan_opts* opts, ficgcn_plan** out);
void ficgcn_plan_destroy(ficgcn_plan* plan);
/* The node order: pi_out[v] = slot of node v inside a column block (the
 * client packs its inputs in this order, paper App. B). */
ficgcn_status ficgcn_plan_node_order(const ficgcn_plan* plan, int32_t* pi_out);
/* Inter-CA copy structure of layer `layer` (the client builds its encrypted
 * copies from it, paper Sec. 3.3.2): src_out[k * n_v + v] = the node whose
 * features copy k holds at node v's slot, -1 for none; copy 0 is the node
 * itself.  K = info "K". */
ficgcn_status ficgcn_plan_copy_sources(const ficgcn_plan* plan, uint32_t layer, int32_t* src_out);
/* Rotation steps whose keys the client must generate (sorted, in [1, M)). */
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
/* Shifts of layer `layer` (SpIntra-CA), sorted. */
ficgcn_status ficgcn_plan_shifts(const ficgcn_plan* plan, uint32_t layer, int64_t* out, size_t cap, size_t* n_out);
/* Integer weights of a layer as the plan encodes them (round_half_even(w * sW)). */
ficgcn_status ficgcn_plan_weights_int(const ficgcn_plan* plan, uint32_t layer, int64_t* out);
/* Number of plaintext operands of a layer and the slot vector of operand i
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
/* Encodes every operand with the library's encoder.  Synchronous. */
ficgcn_status ficgcn_plan_encode(ckks_ctx* ctx, ficgcn_plan* plan);
/* Installs operand i of a layer from coefficient-form residues [level+1][N]
 * at the operand's level (ficgcn_plan_operand_level), for operands encoded
 * elsewhere. */
ficgcn_status ficgcn_plan_load_operand(ckks_ctx* ctx, ficgcn_plan* plan, uint32_t layer, size_t i,
                                       const uint64_t* host_coeffs);

/* Fills every operand of the plan with uniform residues drawn on the device
 * (ChaCha20 stream (6, layer * 2^20 + operand, limb) of `seed`, one the
 * scheme never uses).  For latency measurement only: the layer runs exactly
 * as with encoded operands, but its words mean nothing. */
ficgcn_status ficgcn_plan_fill_operands(ckks_ctx* ctx, ficgcn_plan* plan, uint64_t seed);

/* Runs layer `layer` of the plan (combination, packing, aggregation,
 * rescales and the x^2 activation as the plan schedules them).
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

/* Enumerates the candidate options for this graph size and model: every
 * feasible t, NOO off (when the graph fits one column block) or on with TH
 * in {64, 256, 1024, 4096} below n_v (plus TH = n_v), families 1, 2 and 4;
 * the other fields are copied from base.  Writes up to cap entries, *n_out =
 * the full count.  Host only. */
ficgcn_status ficgcn_plan_candidates(uint32_t n_v, const uint32_t* dims, uint32_t n_layers, uint32_t log_n,
                                     const ficgcn_plan_opts* base, ficgcn_plan_opts* out, size_t cap,
                                     size_t* n_out);
/* Local-adjacency features of one candidate, computed from the CSR graph
 * (as ficgcn_plan_create takes it) without building the plan: degree
 * statistics, locality of the given node order, shift counts of the
 * identity order, and the candidate's t, B, TH, family.  Host only; out
 * holds FICGCN_N_FEATURES floats. */
ficgcn_status ficgcn_candidate_features(const int32_t* rowptr, const int32_t* col, uint32_t n_v, const uint32_t* dims,
                                        uint32_t n_layers, uint32_t log_n, const ficgcn_plan_opts* opts, float* out);
/* Analytic judge: algorithmic HBM bytes of one batched inference of the
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

/* Picks the options of the plan to build.  model == NULL: exhaustive
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
 * Continuous batching of encrypted GCN inferences on one GPU.  The server
 * runs up to n_slots requests at once, each on its own context and stream
 * (so their kernels overlap on the device), admits waiting requests in FIFO
 * order as slots and device memory free up (a later request that fits may
 * pass the head until the head has been passed 16 times), and keeps every
 * client's evaluation keys resident (the caller's ckks_keys objects).  A
 * request's footprint = its input ciphertexts + every layer's outputs + its
 * encoded plan operands; it must fit under hbm_budget_bytes next to the
 * running requests (per-slot scratch is outside the budget). */
typedef struct ficgcn_server ficgcn_server;

typedef struct {
  const ficgcn_plan* plan;         /* the graph's plan (server side); serves one request at a time */
  const ckks_keys* eval_keys;      /* the client's keys, resident on the device */
  const uint64_t* inputs_host;     /* n_in client ciphertexts [n_in][2][level_in+1][N] in host memory
                                      (pinned for an asynchronous upload); read while the request runs */
  size_t n_in;
  uint64_t* output_host;           /* the last layer's n_out ciphertexts [n_out][2][level_out+1][N] */
  size_t n_out;
} ficgcn_request;

typedef struct {
  int32_t status;                  /* the request's ficgcn_status */
  double queue_ms, run_ms, latency_ms;   /* submission to admission, admission to completion, total */
  uint64_t footprint_bytes;
} ficgcn_request_result;

typedef struct {
  uint32_t completed, failed;
  double p50_ms, p99_ms, mean_ms;  /* latency (submission to completion), nearest-rank percentiles */
  double throughput_per_s;         /* completed requests / (last completion - first submission) */
  uint64_t peak_bytes;             /* largest admitted footprint sum */
  uint32_t max_concurrent;         /* most requests running at once */
} ficgcn_server_summary;

/* Creates the slots (contexts for params on the current device, one stream
 * each, at the default priority) and their worker threads. */
ficgcn_status ficgcn_server_create(const ckks_params* params, uint32_t n_slots, uint64_t hbm_budget_bytes,
                                   ficgcn_server** out);
/* Stops the workers after their running requests; waiting requests are dropped. */
void ficgcn_server_destroy(ficgcn_server* server);
/* Queues a request; ENOMEM if it can never fit the budget, EINVAL if its plan
 * has other parameters or another request of the same plan is pending. */
ficgcn_status ficgcn_server_submit(ficgcn_server* server, const ficgcn_request* req, uint64_t* id_out);
/* Blocks until the request completes; returns its status. */
ficgcn_status ficgcn_server_wait(ficgcn_server* server, uint64_t id, ficgcn_request_result* out);
ficgcn_status ficgcn_server_stats(ficgcn_server* server, ficgcn_server_summary* out);

#ifdef __cplusplus
}
#endif
#endif
