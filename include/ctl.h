/*
 * ctl.h — C ABI of libcryptotl: the server-side hot path of CryptoTL's encrypted frozen-layer
 * forward pass (RNS-CKKS) on one AMD Instinct MI355X (gfx950), plus the client-side calls that
 * feed and read it.
 *
 * The paper's protocol (CryptoTL, Section 3, the Train/Classify protocol figure) has the client
 * hold a key pair and encrypt with HE.Enc_pk, the server evaluate ClassifyHE(c, M_S) on its frozen
 * layers, and the client decrypt with HE.Dec_sk. The calls below follow that split:
 *
 *   client:  ctl_keygen, ctl_encode / ctl_encode_items, ctl_encrypt / ctl_encrypt_sym,
 *            ctl_decrypt, ctl_decode*, ctl_ct_pack / ctl_ct_unpack (wire format)
 *   server:  ctl_model_load*, ctl_dense, ctl_square, ctl_replicate, ctl_rescale, ctl_rotate,
 *            ctl_forward  (= ClassifyHE)
 *
 * Conventions
 *   - Every call returns int: CTL_OK (0) or a negative CTL_E* code. ctl_last_error() returns a
 *     thread-local message for the last failure. No C++ exception crosses the ABI.
 *   - On error, outputs are left unchanged and inputs are never modified.
 *   - Handles (ctl_ctx, ctl_sk, ctl_pk, ctl_evk, ctl_model) are owned by the library; free each
 *     with its ctl_*_free call. Device buffers passed as uint64_t* are owned by the caller.
 *   - Ciphertext batches are caller-owned device buffers of uint64 residues in NTT form
 *     (bit-reversed evaluation order: slot i holds a(psi^{2 brv(i) + 1})), laid out
 *     [n_ct][2][k][N] — ciphertext, polynomial (c0, c1), prime q_0..q_{k-1}, coefficient.
 *     k = level + 1 is the number of live primes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the device's default stream). Device calls
 *     are enqueued asynchronously on it. Calls that return host data synchronize it first.
 *   - One context may be used by one stream at a time: calls that overlap on the same context
 *     share its workspace and race.
 *   - Key and model handles may be used with any context of identical parameters on the same
 *     device (several contexts, one per stream, can serve one parameter set with shared keys and
 *     banks); a handle from a context of other parameters is rejected with CTL_EINVAL.
 *   - ctl_ctx_free may come before the frees of handles made on that context, in any order: it
 *     releases the context's workspace at once, and the context's tables go with the last of its
 *     handles. Its allocator hook (ctl_set_allocator) must stay callable until then, since
 *     freeing those handles returns their device memory through it. A context may not be used
 *     after ctl_ctx_free; its handles may, with other contexts of identical parameters.
 *
 * Readings of what the paper leaves open (prime choice, NTT order, slot order, sampling, key
 * switching variant, rounding) are listed in the design notes; the integer results of every
 * call are defined exactly by them and are bit-reproducible across runs.
 */
#ifndef CTL_H
#define CTL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define CTL_OK 0
#define CTL_EINVAL -1    /* bad argument (null pointer, size, layout) */
#define CTL_ENOMEM -2    /* device or host allocation failed */
#define CTL_ELEVEL -3    /* modulus chain exhausted / wrong level for this call */
#define CTL_ESCALE -4    /* encoded value or scale out of range */
#define CTL_EKEY -5      /* a needed Galois or relinearization key is missing */
#define CTL_EHIP -6      /* HIP runtime error */
#define CTL_EPARAM -7    /* no suitable prime / unsupported parameter set */

#define CTL_MAX_PRIMES 8    /* ciphertext primes per chain (the special prime comes on top) */

/* Thread-local text of the last error. Valid until the next failing call on this thread. */
const char *ctl_last_error(void);

/* ------------------------------------------------------------------ parameters */
/* CKKS parameter set ("The CKKS HE scheme" and "Multiplicative Depth", Section 3.1): ring degree
 * N = 2^log2n (supported: 12, 13, 14), ciphertext primes q_0..q_{n_q-1} of the given bit sizes
 * (each prime = 1 mod 2N, the largest such prime below 2^bits not already taken, in listed order),
 * one special key-switching prime P of p_bits (chosen last), default scale 2^log2_scale, and the
 * standard deviation of the discrete Gaussian error. Bit sizes must lie in [log2n + 2, 61]. */
typedef struct ctl_params {
    int log2n;
    int n_q;
    int q_bits[CTL_MAX_PRIMES];
    int p_bits;
    int log2_scale;
    double sigma;
} ctl_params;

/* Host only (no device needed): the primes q_0..q_{n_q-1}, P of a parameter set.
 * primes_out: host array of at least n_q + 1 entries; *n_out receives n_q + 1. */
int ctl_params_primes(const ctl_params *params, uint64_t *primes_out, int *n_out);

/* Host only: the Galois element 5^(r mod N/2) mod 2N of a left rotation by r slots (SIMD
 * Encoding, Section 3.1: rot_r rotates the slot vector r steps to the left; r < 0 rotates right). */
int ctl_galois_elt(const ctl_params *params, int rotation, uint64_t *g_out);

/* Host only: the client-side sampler, exposed so tests can check it. Draws n values from the
 * ChaCha20 (RFC 8439) stream keyed by `seed` with nonce (tag, index): kind 0 = ternary {-1,0,1},
 * kind 1 = discrete Gaussian (|e| <= 19), kind 2 = uniform residues mod `modulus`. out: host int64[n]. */
int ctl_sample(const ctl_params *params, uint64_t seed, uint32_t tag, uint64_t index, int kind,
               uint64_t modulus, int n, int64_t *out);

/* ------------------------------------------------------------------ context */
typedef struct ctl_ctx ctl_ctx;

/* Create a context on HIP device `device`: derives the primes and NTT tables and uploads them. */
int ctl_ctx_create(const ctl_params *params, int device, ctl_ctx **ctx_out);
int ctl_ctx_free(ctl_ctx *ctx);
/* primes_out: host array of n_q + 1 entries (q_0..q_{n_q-1}, P); *n_out = n_q + 1. */
int ctl_ctx_primes(const ctl_ctx *ctx, uint64_t *primes_out, int *n_out);

/* Launch knobs an autotuner may set per context. They change which kernels run and how their
 * work is divided, never the results (every choice computes the same residues):
 *   CTL_KNOB_MAC_CHUNK   largest number of giant-step accumulators a MAC thread keeps (1..16,
 *                        default 16; the chunk used is the largest of 16, 12, 8, 6, 4, 3, 2, 1
 *                        that divides t2 and does not exceed this cap);
 *   CTL_KNOB_MAC_CTS     ciphertexts per MAC workgroup, sharing its staged plaintexts (1..16,
 *                        default 16; the integer-prime MAC takes at most 8);
 *   CTL_KNOB_KEYIP_XCD   1 (default): key-product workgroups numbered so that all rotations of a
 *                        digit tile run on one XCD; 0: tiles first;
 *   CTL_KNOB_MAC_DIRECT  largest batch whose MAC reads plaintext words directly instead of staging
 *                        them in LDS for the workgroup's ciphertexts (0..64, default 3: at N = 2^14
 *                        the direct form is faster up to 3 ciphertexts, the staged one from 4);
 *   CTL_KNOB_NTT_XCD     1 (default): ModUp workgroups numbered so that the targets of one digit,
 *                        and ModDown workgroups so that the primes of one group, run on one XCD
 *                        and share its L2; 0: plain order;
 *   CTL_KNOB_MAC_LIMB    1 (default): the plaintext MAC and the key product over primes of 41..60
 *                        bits multiply 30-bit limbs into carry-free column sums (the MAC then
 *                        keeps at most 8 giant-step accumulators per thread); 0: 128-bit
 *                        accumulation. Primes of 61 bits always take the latter;
 *   CTL_KNOB_KEYIP_RR    hoisted rotations per key-product workgroup, which read each digit word
 *                        once for all of them (1..8, default 8; 5 and 7 act as 4 and 6; each
 *                        arithmetic class caps it by its register budget, e.g. 8 for FP64 rows
 *                        and 4 for 30-bit-limb rows with 6 primes, 1 for limb rows with 8;
 *                        launches over at most 4 ciphertexts use at most 2; launches whose
 *                        rotations have their own digits use 1);
 *   CTL_KNOB_NTT_SPLIT   launches of fewer residue transforms than this (0..4096, default 128; 0:
 *                        never) split every transform over N/1024 single-wave workgroups in two
 *                        launches through a workspace buffer, instead of one workgroup per
 *                        transform (small batches fill the GPU; same residues);
 *   CTL_KNOB_NTT_LOOP    launches with at least this many residue transforms per compute unit
 *                        in each arithmetic class present, FP64 primes and integer primes
 *                        (0..64, default 8; 0: never), run as resident workgroups that loop
 *                        over the transforms of one class per launch, bringing the next one's
 *                        input into L2 while they compute the current one (same residues);
 *   CTL_KNOB_FUSE_RESCALE 1 (default): the ModDown by P that ends a key switch and the rescale
 *                        after it (dense layers, products) run as one pass: the inverse transforms
 *                        of the last prime's row and the P row, then one forward transform per
 *                        remaining prime (same residues); 0: the two steps apart.
 * Out-of-range values give CTL_EINVAL and leave the knob unchanged. */
#define CTL_KNOB_MAC_CHUNK 0
#define CTL_KNOB_MAC_CTS 1
#define CTL_KNOB_KEYIP_XCD 2
#define CTL_KNOB_MAC_DIRECT 3
#define CTL_KNOB_NTT_XCD 4
#define CTL_KNOB_MAC_LIMB 5
#define CTL_KNOB_KEYIP_RR 6
#define CTL_KNOB_NTT_SPLIT 7
#define CTL_KNOB_NTT_LOOP 8
#define CTL_KNOB_FUSE_RESCALE 9
int ctl_knob_set(ctl_ctx *ctx, int knob, int value);
int ctl_knob_get(const ctl_ctx *ctx, int knob, int *value);

/* Optional device allocator for the context's workspace and the key and model banks (for example
 * the framework's caching allocator). alloc returns a device pointer of at least `bytes` bytes
 * usable on `stream`, or NULL. Without a hook the library uses hipMalloc / hipFree. Install it
 * before any allocation is made. */
typedef void *(*ctl_alloc_fn)(uint64_t bytes, void *stream, void *user);
typedef void (*ctl_free_fn)(void *ptr, void *stream, void *user);
int ctl_set_allocator(ctl_ctx *ctx, ctl_alloc_fn alloc, ctl_free_fn free_fn, void *user);

/* Bytes of device workspace the context currently holds (grows on demand, freed with the ctx). */
int ctl_workspace_bytes(const ctl_ctx *ctx, uint64_t *bytes_out);

/* Freeze (frozen = 1) or unfreeze the workspace. While frozen the workspace never moves: a call that
 * would need more of it fails with CTL_ENOMEM instead of reallocating. Freeze after a first run of
 * the largest shapes before capturing launch sequences into a HIP graph, so that captured graphs
 * never refer to freed workspace. */
int ctl_workspace_freeze(ctl_ctx *ctx, int frozen);

/* Forward (inverse = 0) or inverse (inverse = 1) negacyclic NTT, in place, of n_res residue
 * polynomials of N words each, stored back to back at device pointer `dev`. prime_idx: host
 * array of n_res prime indices (0..n_q-1 for q_i, n_q for P). Values must be < their prime. */
int ctl_ntt(ctl_ctx *ctx, uint64_t *dev, int n_res, const int32_t *prime_idx, int inverse,
            void *stream);

/* Parity hooks (the bit-exact tests feed both the library and an independent implementation the
 * same integers, since FP64 encoding is not bit-reproducible across implementations).
 * Residue polynomials [n_poly][k][N] over q_0..q_{k-1} (a ciphertext has n_poly = 2), in NTT form
 * (CTL_FORM_NTT, the library's form at rest) or coefficient form (CTL_FORM_COEFF).
 * ctl_ct_export copies device `ct` (NTT form) to host `host_out`, transformed to the requested
 * form on the device first; synchronizes the stream. ctl_ct_import copies host residues in the given
 * form to device `ct_out` in NTT form; every word must be reduced modulo its row's prime, else
 * CTL_EINVAL and nothing is written; synchronizes. ctl_pt_import uploads n_pt signed integer
 * plaintexts (host int64 [n_pt][N] coefficients, |c| < 2^62, else CTL_ESCALE) to device `pt_out` as
 * [n_pt][k][N] NTT form over q_0..q_{k-1}, or [n_pt][k+1][N] with a last row mod P when ext != 0
 * (the layout of a plaintext-bank row of a layer with baby steps over Q*P); synchronizes. k outside
 * 1..n_q gives CTL_ELEVEL. */
#define CTL_FORM_NTT 0
#define CTL_FORM_COEFF 1
int ctl_ct_export(ctl_ctx *ctx, const uint64_t *ct, int k, int n_poly, int form, uint64_t *host_out,
                  void *stream);
int ctl_ct_import(ctl_ctx *ctx, const uint64_t *host, int k, int n_poly, int form, uint64_t *ct_out,
                  void *stream);
int ctl_pt_import(ctl_ctx *ctx, const int64_t *coeffs, int n_pt, int k, int ext, uint64_t *pt_out,
                  void *stream);

/* Instrumentation for benchmarks: while enabled, every kernel launch the context makes is
 * bracketed by a pair of HIP events recorded on the launch stream. ctl_profile_read synchronizes
 * the recorded events and returns, for kernel family `family` (0 .. ctl_profile_families()-1),
 * the number of launches, their summed durations in milliseconds, and the algorithmic work they
 * processed since profiling was enabled: for the NTT-bearing kernels (k_ntt_fwd, k_ntt_inv,
 * k_modup, k_drop, k_int_ntt; a looped launch records its FP64-prime kernel under the same name
 * with an _fp suffix) the number of length-N residue transforms; for the product kernels
 * (k_keyip, k_keyip_fp, k_mac, k_mac_fp, k_mac_direct, k_tensor) the number of 64-bit modular
 * products; for k_add_terms the number of
 * residue words written. fp_work_out receives the part of that work done on primes below 2^41,
 * which run in exact FP64 arithmetic (the rest runs in 64-bit integer arithmetic). Enabling clears
 * earlier records. Adds a few microseconds per launch. */
int ctl_profile_enable(ctl_ctx *ctx, int enable);
int ctl_profile_families(void);
const char *ctl_profile_family_name(int family);
int ctl_profile_read(ctl_ctx *ctx, int family, int *launches_out, double *total_ms_out,
                     double *work_out, double *fp_work_out);
/* Algorithmic HBM bytes of the launches of family `family` recorded since profiling was enabled,
 * for the families that model them (k_keyip and k_keyip_fp, each over the residue rows of its
 * arithmetic class: digit words once per ciphertext when the rotations are hoisted, else once per
 * rotation, each key set's key words once, output words, fold words;
 * the MAC families: ciphertext and rotated-ciphertext words once, plaintext-bank words once,
 * output words); 0 for the others. No synchronization. */
int ctl_profile_read_bytes(ctl_ctx *ctx, int family, double *bytes_out);

/* Launch records since profiling was enabled, in launch order: *n_out of them. Record i gives the
 * kernel family, its duration in milliseconds (synchronizes its stop event), algorithmic work and
 * the part on FP64 primes (as ctl_profile_read), algorithmic HBM bytes (as ctl_profile_read_bytes,
 * 0 where not modelled) and the call site: the layer of the model (-1 outside a model's forward
 * pass) and the phase within it ("baby steps", "mac", "giant steps", "moddown", "rescale",
 * "square", "cubic", "replicate"; "" elsewhere; a static string). */
int ctl_profile_launches(ctl_ctx *ctx, int *n_out);
int ctl_profile_launch(ctl_ctx *ctx, int i, int *family_out, double *ms_out, double *work_out, double *fp_work_out,
                       double *bytes_out, int *layer_out, const char **phase_out);

/* Issue-rate probe of the vector ALU, for rooflines: a kernel of `iters` iterations of independent
 * chains of one instruction class runs on every CU (enough waves to fill them) and
 * *lane_ops_out receives lane-operations per second measured with HIP events on `stream`
 * (synchronizes it). kind: 0 = 32-bit integer add, 1 = 32-bit multiply (low half), 2 = 32 x 32 + 64
 * -> 64-bit multiply-add (v_mad_u64_u32), 3 = FP64 fused multiply-add. */
#define CTL_PROBE_ADD32 0
#define CTL_PROBE_MUL32 1
#define CTL_PROBE_MAD64 2
#define CTL_PROBE_FMA64 3
int ctl_probe_valu(ctl_ctx *ctx, int kind, int iters, double *lane_ops_out, void *stream);

/* ------------------------------------------------------------------ keys (client side) */
typedef struct ctl_sk ctl_sk;
typedef struct ctl_pk ctl_pk;
typedef struct ctl_evk ctl_evk;

/* Key generation from a seed (the protocol's key pair (sk, pk), Section 3): ternary secret s,
 * public key (-a s + e, a) over q_0..q_L, one Galois key per distinct rotation amount in
 * `rotations` (host int32[n_rot]; duplicates and 0 are ignored) and, if relin != 0, a
 * relinearization key. Keys use one digit per ciphertext prime and the special prime P.
 * Any of sk_out / pk_out / evk_out may be NULL if not wanted. Blocks until done. */
int ctl_keygen(ctl_ctx *ctx, uint64_t seed, const int32_t *rotations, int n_rot, int relin,
               ctl_sk **sk_out, ctl_pk **pk_out, ctl_evk **evk_out);
int ctl_sk_free(ctl_sk *sk);
int ctl_pk_free(ctl_pk *pk);
int ctl_evk_free(ctl_evk *evk);
/* Export for checking: sk as int64[N] ternary coefficients; pk as uint64[2][n_q][N] NTT form;
 * the key of Galois element g (g = 0 selects the relinearization key) as uint64[n_q][2][n_q+1][N]
 * (digit, polynomial b/a, prime q_0..q_{n_q-1},P, coefficient), NTT form. Host buffers. */
int ctl_sk_export(const ctl_sk *sk, int64_t *coeffs_out);
int ctl_pk_export(const ctl_pk *pk, uint64_t *out);
int ctl_evk_export(const ctl_evk *evk, uint64_t galois_elt, uint64_t *out);
/* Number of Galois keys held and their elements (host uint64 array of at least that many). */
int ctl_evk_galois(const ctl_evk *evk, uint64_t *elts_out, int *n_out);
/* Evaluation keys as a server receives them from a client (the protocol of Section 3 has the
 * client hold the key pair; the server needs only these public keys to evaluate): n_keys keys,
 * key i for Galois element galois_elts[i] (0 = relinearization key) in host array keys[i] with the
 * export layout above. Every element must be 0 or an odd rotation element below 2N, with no
 * duplicates, and every word must be reduced modulo the prime of its row; otherwise CTL_EINVAL
 * and nothing is allocated. Copies the keys to device memory and blocks until done. */
int ctl_evk_import(ctl_ctx *ctx, const uint64_t *galois_elts, int n_keys, const uint64_t *const *keys,
                   ctl_evk **evk_out);
/* Device bytes held by a key set / by a model's plaintext banks. */
int ctl_evk_bytes(const ctl_evk *evk, uint64_t *bytes_out);

/* ------------------------------------------------------------------ model (server side) */
#define CTL_ACT_NONE 0
#define CTL_ACT_SQUARE 1

/* Degree-3 polynomial activation c0 + c1 z + c2 z^2 + c3 z^3 (coef of the layer descriptor), the
 * form of the paper's ReLU approximation (Section 3.1, "ReLU"); depth 2. */
#define CTL_ACT_POLY3 2

/* Layer kinds (Section 3.1):
 *   CTL_LAYER_DENSE    y = W x by Eq. (1); weights [n_out][n_in]; t1 = BSGS baby steps.
 *   CTL_LAYER_CONV1D   packed single-channel 1D convolution ("1D Convolutions"), filter size f
 *                      (odd), 'same' zero padding, n_out = n_in; y[s] = sum_i w_i x[s + i - (f-1)/2];
 *                      weights [f]; f plaintext products, f - 1 rotations.
 *   CTL_LAYER_AVGPOOL  average pooling, stride 1, size f ("Average Pool"), n_out = n_in - f + 1;
 *                      sum_{i < f} rot_{-i}(x) times a plaintext holding 1/f on the valid
 *                      outputs; no weights. Its outputs sit at slots f-1 .. n_in-1 of each block,
 *                      and the layer that follows (which must be dense) reads them there. */
#define CTL_LAYER_DENSE 0
#define CTL_LAYER_CONV1D 1
#define CTL_LAYER_AVGPOOL 2

/* Giant-step variant of a dense layer: by default every giant-step rotation is a full key switch
 * with its own ModDown; with CTL_LAYER_LAZY_GIANT the key products of all giant steps are summed
 * over Q*P and lowered by a single ModDown (same value up to rounding, one rounding instead of
 * t2 - 1, about 40% fewer residue transforms in the ModDown kernels). */
#define CTL_LAYER_LAZY_GIANT 1
/* Baby steps kept over Q*P ("double hoisting", Bossuat et al., Eurocrypt 2021): each baby-step
 * rotation of a dense layer stays in the extended basis (its key product plus P sigma_j(c0), no
 * ModDown), the diagonal plaintexts are stored with a residue mod P as well, the products of
 * Eq. (1) are summed over Q*P, and only the c1 of each giant step and the final sum are lowered:
 * t2 + 1 polynomials per ciphertext go through ModDown instead of 2 t1. Implies
 * CTL_LAYER_LAZY_GIANT. Same value up to rounding; the bank takes (k+1)/k of the memory. Also
 * for convolutions and average pools: their rotations over Q*P, one ModDown of the sum. */
#define CTL_LAYER_BABY_QP 2

/* One layer. A dense layer y = W x with W of shape [n_out][n_in] is evaluated by the baby-step
 * giant-step diagonal method (Eq. (1) of Section 3.1) with padded width t = max(off + n_in, n_out),
 * t = t1 * t2 (t1 must divide t; off = f - 1 after an average pool, else 0). act applies x^2
 * (CTL_ACT_SQUARE) or the cubic in coef (CTL_ACT_POLY3) after the layer, never after the last.
 * flags: 0, CTL_LAYER_LAZY_GIANT (dense only) or CTL_LAYER_BABY_QP. Zero-filled fields select a
 * dense layer. */
typedef struct ctl_layer_desc {
    int n_in;
    int n_out;
    int t1;          /* dense: baby steps (divides the padded width) */
    int act;         /* CTL_ACT_* applied after the layer (not after the last) */
    int flags;       /* CTL_LAYER_LAZY_GIANT, CTL_LAYER_BABY_QP */
    int kind;        /* CTL_LAYER_* */
    int f;           /* conv / pool size */
    double coef[4];  /* CTL_ACT_POLY3: c0..c3 */
} ctl_layer_desc;

typedef struct ctl_model ctl_model;

/* Plan summary of a loaded model. Slot layout ("Multiple Predictions", Section 3.1): each item
 * occupies a block of `block` = 2 t_max slots; items = floor((N/2) / block) items per ciphertext.
 * The input ciphertext must be at k_in = n_q primes with scale scale_in; the output has k_out
 * primes and scale scale_out. */
typedef struct ctl_model_info {
    int n_layers;
    int block;
    int items;
    int k_in;
    int k_out;
    int n_in;
    int n_out;
    int n_rotations;
    double scale_in;
    double scale_out;
    int layer_k[8];      /* live primes at each layer's input */
    int layer_t[8];      /* padded width t of each layer */
} ctl_model_info;

/* Plan overrides for models that share one slot layout or start below the top level (used when
 * several models serve one batch, e.g. layers of different widths at different depths): block =
 * slot stride per item (0: 2 t_max of this model; else at least 2 t_max and at most N/2); k_in =
 * live primes at the first layer's input (0: all n_q); scale_in = input scale (0: 2^log2_scale). */
typedef struct ctl_model_opts {
    int block;
    int k_in;
    double scale_in;
} ctl_model_opts;

/* Load a model from FP64 weights (weights != NULL) or from already-encoded integer plaintexts
 * (pts != NULL; exactly one of the two), with optional plan overrides (opts may be NULL). The
 * other two load calls are this one with opts = NULL. */
int ctl_model_load_ex(ctl_ctx *ctx, const ctl_layer_desc *layers, int n_layers,
                      const double *const *weights, const int64_t *const *pts,
                      const ctl_model_opts *opts, ctl_model **model_out);

/* Load the frozen layers from FP64 weights: for a dense layer W[l] is a host row-major
 * [n_out][n_in] matrix, for a convolution the f taps, for an average pool it is ignored (may be
 * NULL). The plaintexts (diag'_i of Eq. (1), the masked taps, the pooling mask) are encoded at the
 * scale of the prime each layer's rescale drops, reduced and transformed on the device, and kept
 * resident in HBM. Before a dense layer or a convolution whose input is not already [x | x] the
 * forward pass replicates it (ct + rot_{-t}(ct)). */
int ctl_model_load(ctl_ctx *ctx, const ctl_layer_desc *layers, int n_layers,
                   const double *const *weights, ctl_model **model_out);
/* Same, from already-encoded integer plaintexts: pts[l] is a host int64 array of signed
 * coefficients (|c| < 2^62) — dense: [t][N], plaintext i = diag'_i; convolution: [f][N], plaintext
 * i multiplies rot_{i-(f-1)/2}; average pool: [1][N], the pooling plaintext. */
int ctl_model_load_raw(ctl_ctx *ctx, const ctl_layer_desc *layers, int n_layers,
                       const int64_t *const *pts, ctl_model **model_out);
int ctl_model_free(ctl_model *model);
int ctl_model_get_info(const ctl_model *model, ctl_model_info *info_out);
/* Every left-rotation amount the model needs keys for (host int32 array of n_rotations). */
int ctl_model_rotations(const ctl_model *model, int32_t *rots_out, int *n_out);
int ctl_model_bytes(const ctl_model *model, uint64_t *bytes_out);

/* ------------------------------------------------------------------ client encode / encrypt */
/* Encode N/2 real slot values at `scale` into signed integer plaintext coefficients:
 * m = rint(scale * tau^{-1}(z)) with slot j <-> zeta^{5^j}, zeta = exp(i pi / N). Host buffers:
 * slots double[N/2], coeffs_out int64[N]. CTL_ESCALE if a coefficient reaches 2^62. */
int ctl_encode(ctl_ctx *ctx, const double *slots, double scale, int64_t *coeffs_out);
/* Place `items` feature vectors x (host double [items][n_in]) as [x | x] blocks of the model's
 * layout and encode them at the model's input scale into coeffs_out (host int64[N]). */
int ctl_encode_items(ctl_ctx *ctx, const ctl_model *model, const double *x, int items,
                     int64_t *coeffs_out);
/* Public-key encryption at the top level (HE.Enc_pk): ct = (v b + e0 + m, v a + e1) with v ternary
 * and e0, e1 Gaussian drawn from `seed`. coeffs: host int64[N] plaintext coefficients;
 * ct_out: device uint64[2][n_q][N]. */
int ctl_encrypt(ctl_ctx *ctx, const ctl_pk *pk, const int64_t *coeffs, uint64_t seed,
                uint64_t *ct_out, void *stream);
/* Seeded secret-key encryption at the top level: ct = (-a s + e + m, a) with a uniform (drawn as
 * NTT values, prime by prime, from the stream (seed, 11, 0)) and e Gaussian (stream (seed, 12, 0)).
 * c1 = a depends on the seed alone, so a client can send c0 and the seed: half the upload, the
 * size Table 2's client-to-server column implies. ct_out: device uint64[2][n_q][N]; blocks. */
int ctl_encrypt_sym(ctl_ctx *ctx, const ctl_sk *sk, const int64_t *coeffs, uint64_t seed,
                    uint64_t *ct_out, void *stream);
/* Server side of a seeded upload: c0 (host uint64[n_q][N], every word reduced, else CTL_EINVAL)
 * and the seed become the full ciphertext at device pointer ct_out ([2][n_q][N]); blocks. */
int ctl_expand_seeded(ctl_ctx *ctx, const uint64_t *c0, uint64_t seed, uint64_t *ct_out, void *stream);
/* Decryption (HE.Dec_sk) of one ciphertext with k live primes at device pointer ct: writes the
 * coefficient-form residues of c0 + c1 s to host uint64[k][N]. Synchronizes the stream. */
int ctl_decrypt(ctl_ctx *ctx, const ctl_sk *sk, const uint64_t *ct, int k, uint64_t *residues_out,
                void *stream);
/* Decode coefficient residues (host uint64[k][N]) at `scale` into N/2 real slots (host double). */
int ctl_decode(ctl_ctx *ctx, const uint64_t *residues, int k, double scale, double *slots_out);
/* Decode a model output: y_out host double [items][n_out] read from slots [b*block, b*block+n_out). */
int ctl_decode_items(ctl_ctx *ctx, const ctl_model *model, const uint64_t *residues, double *y_out);

/* ------------------------------------------------------------------ wire format (host only) */
/* Serialized ciphertexts for the client-server messages (Section 5.1, "Runtime and Data Communication", Table 2:
 * the client sends a ciphertext at the top level, the server returns one at q_0). Little-endian:
 *   bytes 0-3 "CTL1", 4 version (1), 5 log2 N, 6 k, 7 n_poly (2: (c0, c1); 1: c0 of a seeded
 *   symmetric ciphertext), 8-15 FNV-1a-64 digest of the primes q_0..q_{n_q-1}, P as little-endian
 *   words, 16-23 the seed (n_poly = 1) or 0; then for each polynomial and each prime q_i
 *   (i < k) the N residues, each in bits(q_i) bits, least significant bit first, packed
 *   back to back (every row is a whole number of bytes because N is a multiple of 8).
 * Size: 24 + n_poly * N * sum_{i<k} bits(q_i) / 8 bytes. ct: host uint64[n_poly][k][N].
 * Pack fails with CTL_EINVAL on an unreduced word or a short buffer; unpack rejects a wrong magic,
 * version or length (CTL_EINVAL), another parameter set (CTL_EPARAM) or an unreduced word, and
 * then writes nothing. ct_out must hold n_poly * k * N words (at most 2 * n_q * N). */
int ctl_ct_packed_bytes(const ctl_params *params, int k, int n_poly, uint64_t *bytes_out);
int ctl_ct_pack(const ctl_params *params, const uint64_t *ct, int k, int n_poly, uint64_t seed, uint8_t *out,
                uint64_t cap, uint64_t *len_out);
int ctl_ct_unpack(const ctl_params *params, const uint8_t *in, uint64_t len, uint64_t *ct_out, int *k_out,
                  int *n_poly_out, uint64_t *seed_out);

/* ------------------------------------------------------------------ server hot path (batched) */
/* All take n_ct ciphertexts [n_ct][2][k][N] at device pointer `in` and write [n_ct][2][k'][N] to
 * device pointer `out` (out must not overlap in). */

/* ClassifyHE (protocol figure, Section 3): every frozen layer in turn — dense, then for all but
 * the last layer x^2 with relinearization and rescale, then replicate [y | 0] -> [y | y] for the
 * next layer. in: k = model k_in; out: k = model k_out. */
int ctl_forward(ctl_ctx *ctx, const ctl_model *model, const ctl_evk *evk, const uint64_t *in,
                uint64_t *out, int n_ct, void *stream);

/* ctl_forward on a batch that mixes clients (ClassifyHE of the protocol figure of Section 3, for
 * several key owners at once): ciphertext b is evaluated with evks[b], an array of n_ct handles (host memory, read during
 * the call only). Consecutive equal handles form a run; the key products of Section 3.1's
 * rotations and relinearizations run once per run, every other kernel (NTTs, ModUp, ModDown,
 * plaintext products, rescales) once over the whole batch. Output b equals ctl_forward of
 * ciphertext b alone with evks[b], bit for bit. Errors: a NULL handle or one of other parameters
 * gives CTL_EINVAL; a handle without a key the model needs gives CTL_EKEY. */
int ctl_forward_multi(ctl_ctx *ctx, const ctl_model *model, const ctl_evk *const *evks,
                      const uint64_t *in, uint64_t *out, int n_ct, void *stream);

/* One layer of the model. Dense, by Eq. (1): hoisted baby-step rotations rot_j, j < t1, products
 * with the diagonal plaintexts, one key switch per giant step rot_{k t1}, one rescale at the end.
 * Convolution and average pool: their rotations hoisted the same way, the plaintext products
 * summed, one rescale. The input must already be in the layer's layout (the replicate that
 * ctl_forward inserts is not part of this call). in: k = ctl_model_info.layer_k; out: k - 1. */
int ctl_dense(ctl_ctx *ctx, const ctl_model *model, int layer, const ctl_evk *evk,
              const uint64_t *in, uint64_t *out, int n_ct, void *stream);

/* Dense layers of several models over one batch grouped by model (queries whose layers have
 * different widths, evaluated together): group g is counts[g] consecutive ciphertexts of `in`
 * (n_ct = the sum of counts), evaluated by layer `layer` of models[g] exactly as ctl_dense of that
 * model and layer alone would, bit for bit. Every such layer must keep its baby steps over Q*P
 * (CTL_LAYER_BABY_QP; else CTL_EINVAL) and start at the same level k (else CTL_ELEVEL); the
 * models may differ in width, t1 and t2 but must share one slot layout to be useful together.
 * The hoisted ModUp of every ciphertext (Eq. (1)'s baby steps), the ModUp of every giant step's
 * operand, the final ModDown and the rescale each run once over the whole batch; the key
 * products, the plaintext products and the giant-step sums run per group. models, counts: host
 * arrays of n_groups entries (1..4096). in: [n_ct][2][k][N]; out: [n_ct][2][k-1][N]. A missing
 * Galois key of any group gives CTL_EKEY before anything is enqueued. */
int ctl_dense_groups(ctl_ctx *ctx, const ctl_model *const *models, const int *counts, int n_groups, int layer,
                     const ctl_evk *evk, const uint64_t *in, uint64_t *out, void *stream);

/* Product of two ciphertexts at k primes: tensor, relinearization, rescale. k -> k - 1. */
int ctl_mul(ctl_ctx *ctx, const ctl_evk *evk, int k, const uint64_t *a, const uint64_t *b, uint64_t *out,
            int n_ct, void *stream);

/* Degree-3 activation c0 + c1 z + c2 z^2 + c3 z^3 (coef[0..3]; the paper's ReLU approximation of
 * Section 3.1 has this form) on ciphertexts at k >= 3 primes and scale `scale`, depth 2, k -> k - 2:
 *   z2 = rescale(relin(z z));  u = rescale(z C3) + C2;  w = rescale(relin(z2 u));
 *   v = (rescale(z C1) without its last prime) + C0;   out = w + v,
 * with integer constants rounded (llround) at the scales the terms carry, q_a = q_{k-1},
 * q_b = q_{k-2}: S2 = S S / q_a, S3 = S2 S2 / q_b, C3 = c3 S, C2 = c2 S2, C1 = c1 (S3 q_a / S),
 * C0 = c0 S3 (each product evaluated in this order in FP64). *scale_out receives S3. */
int ctl_poly3(ctl_ctx *ctx, const ctl_evk *evk, int k, double scale, const double *coef, const uint64_t *in,
              uint64_t *out, int n_ct, void *stream, double *scale_out);

/* x^2 activation (the polynomial activation of Section 3.1, degree 2): tensor, relinearize with
 * the relinearization key, rescale. k -> k - 1. */
int ctl_square(ctl_ctx *ctx, const ctl_evk *evk, int k, const uint64_t *in, uint64_t *out,
               int n_ct, void *stream);

/* ct + rot_{-width}(ct): turns [y | 0] blocks into [y | y] for the next layer. k -> k. */
int ctl_replicate(ctl_ctx *ctx, const ctl_evk *evk, int k, int width, const uint64_t *in,
                  uint64_t *out, int n_ct, void *stream);

/* ctl_square for callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops and harnesses that must not call hipMalloc): the same result as ctl_square, bit for bit,
 * with every intermediate (tensor, ModUp digits, key product, ModDown and rescale rows) in a fixed
 * scratch array of CTL_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on, from
 * the first context created on that GPU until the process ends. The call makes no device
 * allocation and uses no workspace of the context. It needs 8 N (k^2 + 9k + 6) bytes of scratch per
 * ciphertext (12 MiB per ciphertext at N = 2^14, k = 6); a batch that does not fit gives CTL_EINVAL
 * before anything is enqueued. Every call on one GPU shares that GPU's scratch, whatever its
 * context or stream: calls that overlap on one GPU race and must be serialized by the caller. The
 * scratch keeps the last call's contents and needs no clearing: every intermediate is written
 * before it is read. Arguments, layout and the other errors as ctl_square. */
#define CTL_NOALLOC_SCRATCH_BYTES (64ull << 20)
int ctl_square_noalloc(ctl_ctx *ctx, const ctl_evk *evk, int k, const uint64_t *in, uint64_t *out,
                       int n_ct, void *stream);

/* Left rotation by `rotation` slots (needs that Galois key). k -> k. */
int ctl_rotate(ctl_ctx *ctx, const ctl_evk *evk, int k, int rotation, const uint64_t *in,
               uint64_t *out, int n_ct, void *stream);

/* Rescale ("The CKKS HE scheme", Section 3.1): divide by q_{k-1} with rounding. k -> k - 1. */
int ctl_rescale(ctl_ctx *ctx, int k, const uint64_t *in, uint64_t *out, int n_ct, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CTL_H */
