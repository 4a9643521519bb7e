// Launch interface of the HIP kernels (device pointers, plain structs passed by value).
#pragma once

#include "ctl_internal.h"

namespace ctl {

// Residue r of a launch lives at offset (in residues) off + outer * ostride + grp * gstride + e,
// where e = r % per, grp = (r / per) % ngrp, outer = r / (per * ngrp); its prime is prime[e].
struct ResMap {
    int per;
    int ngrp;
    long off;
    long gstride;
    long ostride;
    int prime[kMaxMods];
};

struct Tables {
    const u64 *tw, *tws, *itw, *itws;   // [np][N] each
    const PrimeConst *pc;               // [np]
    const CrossConst *cross;            // [kMaxMods][kMaxMods], entry [i * kMaxMods + j]
    unsigned char host_fp[kMaxMods];    // host copy of pc[i].fp, for launch decisions
    unsigned char host_lt60[kMaxMods];  // prime i below 2^60 (30-bit limb products apply)
    int cus;                            // compute units of the device
    int lds_cu;                         // LDS bytes per compute unit
};

constexpr int kMaxKeysPerLaunch = 64;

struct DropAdd {
    const u64 *base;     // addend (NTT form) or null
    long sb, sr, sc;     // strides in words for batch index b, group r, polynomial c
    int R;               // groups per ciphertext (<= kMaxKeysPerLaunch)
    int mask;            // bit c set: add to polynomial c
    u64 gal[kMaxKeysPerLaunch];   // automorphism applied to the addend of group r (1 = none)
};

// Entry y of a launch over residues: idx[y] is the residue row (or, for k_int_ntt, the prime
// index); prime[y] is the prime-table index of that row where a kernel needs both.
struct PrimeList {
    int n;
    int idx[kMaxMods];
    int prime[kMaxMods];
};

// Term folded into the key product of polynomial 0 (see keyip_body): rows t < rows add
// mul[t] * src[b sb + r sr + t N + sigma_r(n)].
struct KeyFold {
    const u64 *src;      // null: no fold
    long sb, sr;
    int rows;
    u64 mul[kMaxMods];
};

// Location of group g of a ModDown input: off + (g / R) sb + (g % R) sr (words).
struct GrpMap {
    long off, sb, sr;
    int R;
};

struct KeyList {
    const u64 *key[kMaxKeysPerLaunch];   // [nq][2][np][N] each
    u64 gal[kMaxKeysPerLaunch];          // Galois element applied to the digits (1 = none)
    u64 ginv[kMaxKeysPerLaunch];         // its inverse mod 2N
};

struct GalList {
    u64 g[kMaxKeysPerLaunch];
};

hipError_t kernels_prepare(int logn);
// Device address of the library's fixed scratch array (kScratchWords words; one copy per GPU,
// held until the process ends) on the current device. Looked up once per device and cached;
// call it with the device current. Used by the entry point that allocates nothing.
constexpr size_t kScratchWords = (size_t)CTL_NOALLOC_SCRATCH_BYTES / 8;
hipError_t scratch_device_address(int device, u64 **out);
// Vector ALU issue-rate probe (kind 0..3, see ctl_probe_valu): `blocks` workgroups of 256 threads,
// each thread 8 chains x 8 steps x iters operations; out: blocks * 256 words.
constexpr int kProbeOpsPerThreadIter = 64;
void launch_probe(int kind, int iters, u64 seed, u64 *out, int blocks, hipStream_t st);
void launch_sum_gather(int logn, u64 *out, long o_sb, const u64 *base, long ba_sb, const u64 *src, long s_sb,
                       long s_sr, int R, int kk, bool ext, int mask, const GalList &gal, int B, int nq,
                       const Tables &tab, hipStream_t st);
// Launch choices an autotuner may set (defaults in brackets): the largest giant-step chunk of the
// MAC [16], ciphertexts per MAC workgroup [8], XCD-grouped key-product numbering [1], largest
// batch that uses the unstaged MAC [3], XCD-grouped ModUp / ModDown numbering [1], 30-bit limb
// products in the integer-prime MAC [1], hoisted rotations per key-product workgroup [8].
struct Knobs {
    int mac_chunk_cap = 16;
    int mac_cts = 8;
    int keyip_xcd = 1;
    int mac_direct_max = 3;      // batches up to this size use the unstaged MAC
    int ntt_xcd = 1;             // XCD-grouped numbering of ModUp and ModDown workgroups
    int mac_limb = 1;            // integer-prime MAC by 30-bit limbs where every prime is below 2^60
    int keyip_rr = 8;            // key product: hoisted rotations per workgroup sharing digit words (1..8)
    int ntt_split = 128;         // launches of fewer transforms split each over N/1024 workgroups (0: never)
    int ntt_loop = 8;            // launches with at least this many transforms of each class per CU loop (0: never)
    int fuse_rescale = 1;        // ModDown by P and the rescale after it as one pass
};

// The NTT-bearing launches: with split_tmp (a buffer of one residue per transform of the launch,
// [count][N] words) every transform is split over N / 1024 single-wave workgroups in two launches,
// for launches of few transforms; launches of many (kn.ntt_loop) run as looped workgroups, one
// kernel per arithmetic class present; otherwise one workgroup per transform. The same residues
// come out of every form. cls (looped launches only): 0 launches the FP64-prime kernel alone, 1
// the integer-prime one, -1 both.
void launch_ntt(int logn, bool inverse, const u64 *in, const ResMap &imap, u64 *out, const ResMap &omap,
                int count, const Tables &tab, const Knobs &kn, hipStream_t st, u64 *split_tmp = nullptr,
                int cls = -1);
void launch_modup(int logn, const u64 *coef, const u64 *d, const ResMap &dmap, u64 *digits, int groups, int k,
                  int nq, const Tables &tab, const Knobs &kn, hipStream_t st, u64 *split_tmp = nullptr,
                  int cls = -1);
void launch_drop(int logn, const u64 *x, const u64 *last, u64 *out, int groups, int k, int drop,
                 const DropAdd &add, const Tables &tab, const Knobs &kn, hipStream_t st,
                 const GrpMap *xmap = nullptr, u64 *split_tmp = nullptr, int cls = -1);
// ModDown by P of groups extended polynomials x (group g, row t at x + g xs + t N; rows 0..kl
// over Q, kl + 1 mod P) followed by the rescale by q_kl, into out ([groups][kl][N]): coef holds
// the inverse transforms of row kl and of the P row ([groups][2][N]); add (R = 1, no rotation)
// must already be folded into row kl by launch_fold_last and is added to rows 0..kl-1 here.
void launch_drop_rescale(int logn, const u64 *x, long xs, const u64 *coef, u64 *out, int groups, int kl, int np,
                         const DropAdd &add, const Tables &tab, const Knobs &kn, hipStream_t st,
                         u64 *split_tmp = nullptr, int cls = -1);
// launch_drop_rescale as a split chain (few polynomials): inverse_part = true launches the
// inverse's wave-local passes over rows kl and P into tmp_i ([2 groups][N]), false the rest
// (tmp_f: [groups kl][N]).
void launch_drop_rescale_chain(int logn, bool inverse_part, const u64 *x, long xs, u64 *out, int groups, int kl, int np,
                               const DropAdd &add, const Tables &tab, hipStream_t st, u64 *tmp_i, u64 *tmp_f);
// x[g][kl] += P a[g][kl] mod q_kl for each group whose polynomial has an addend in add.
void launch_fold_last(int logn, u64 *x, long xs, int groups, int kl, int np, const DropAdd &add, const Tables &tab,
                      hipStream_t st);
// ModUp (iNTT of the digits of d, lifts, NTTs) and ModDown / rescale (iNTT of the dropped prime's
// residue of each group, located by imap; lifts, NTTs and the combine of launch_drop with x, xm,
// add) as split chains, the inverse's top pass fused into the forward top passes:
// inverse_part = true launches the inverse's wave-local passes, false the rest. tmp_i holds one
// residue per inverse transform, tmp_f one per forward transform.
void launch_modup_chain(int logn, bool inverse_part, const u64 *d, const ResMap &dmap, u64 *digits, int groups, int k,
                        int nq, const Tables &tab, hipStream_t st, u64 *tmp_i, u64 *tmp_f);
void launch_drop_chain(int logn, bool inverse_part, const u64 *in, const ResMap &imap, const u64 *x, const GrpMap &xm,
                       u64 *out, int groups, int k, int drop, const DropAdd &add, const Tables &tab, hipStream_t st,
                       u64 *tmp_i, u64 *tmp_f);
// The classes (bit 0: FP64 primes, bit 1: integer primes) that the launch above with the same
// arguments runs as separate looped kernels; 0 when it runs in another form.
int ntt_loop_classes(int count, const ResMap &imap, const Tables &tab, const Knobs &kn, const u64 *split_tmp);
int modup_loop_classes(int groups, int k, int nq, const Tables &tab, const Knobs &kn, const u64 *split_tmp);
int drop_loop_classes(int groups, int k, const Tables &tab, const Knobs &kn, const u64 *split_tmp);
void launch_int_ntt(int logn, const int64_t *src, u64 *out, int groups, const PrimeList &pl,
                    const Tables &tab, hipStream_t st);
// Key products run one launch per arithmetic class of their rows: FP64 products (primes below
// 2^41), 30-bit limbs (below 2^60, with kn.mac_limb) or 128-bit sums.
enum KeyipClass { KIP_FP = 0, KIP_LIMB = 1, KIP_WIDE = 2, KIP_CLASSES = 3 };
// Rows t (0..k; row k is the one mod P) of one key-product launch.
struct RowSet {
    int n;
    int t[kMaxMods];
};
// The rows of a key product over k residues and the special prime, split by class.
void keyip_rows(int k, int nq, const Tables &tab, const Knobs &kn, RowSet (&rows)[KIP_CLASSES]);
// The key product of the rows of one class (see keyip_body); nothing is launched for an empty set.
void launch_keyip(int logn, int k, int cls, const RowSet &rows, const u64 *digits, long db, long dr,
                  const KeyList &keys, int R, u64 *out, long ob, const KeyFold &fold, int B, int nq,
                  const Tables &tab, const Knobs &kn, hipStream_t st);
// rows = k residues per polynomial, or k + 1 with the last one mod P (ext_nq = its prime index;
// -1 without). ct / rot: j = 0 / j >= 1 operands with batch strides ct_sb / rot_sb. part: 0 =
// every row, 1 = the FP64-prime rows only, 2 = the integer-prime rows only (batches above
// kn.mac_direct_max; smaller ones take one unstaged launch over every row whatever part says).
void launch_mac(int logn, const u64 *ct, long ct_sb, const u64 *rot, long rot_sb, const u64 *bank, u64 *inner,
                int B, int rows, int ext_nq, int t1, int t2, const Tables &tab, const Knobs &kn, hipStream_t st,
                int part);
// out[b][c][t] = P x in[b][c][t] mod q_t for t < k, 0 for t = k (the row mod P): in [B][2][k][N],
// out with batch stride o_sb and [2][k+1][N] per ciphertext.
void launch_times_p(int logn, const u64 *in, u64 *out, long o_sb, int B, int k, int nq, const Tables &tab,
                    hipStream_t st);
void launch_add_terms(int logn, const u64 *a, long a_sb, const u64 *terms, long t_sb, long t_ss, int S,
                      u64 *out, int B, int k, const Tables &tab, hipStream_t st);
void launch_tensor(int logn, const u64 *a, const u64 *b, u64 *out, int B, int k, const Tables &tab, hipStream_t st);
// Per-prime constants of k_affine: multiplier (with its Shoup companion floor(mul 2^64 / q)) and
// addend of c0, each reduced mod q_i.
struct AffineConst {
    u64 mul[kMaxMods], muls[kMaxMods], add[kMaxMods];
};
void launch_affine(int logn, const u64 *in, u64 *out, int B, int k_in, int k_out, const AffineConst &ac,
                   const Tables &tab, hipStream_t st);
void launch_ksk_body(int logn, u64 *key, const u64 *e, const u64 *s, u64 g, int nq, const Tables &tab,
                     hipStream_t st);
void launch_pk_body(int logn, u64 *pk, const u64 *e, const u64 *s, int nq, const Tables &tab, hipStream_t st);
void launch_encrypt(int logn, const u64 *pk, const u64 *in, u64 *ct, int nq, const Tables &tab, hipStream_t st);
void launch_dec_mul(int logn, const u64 *ct, const u64 *s, u64 *out, int k, const Tables &tab, hipStream_t st);

}  // namespace ctl
