// C ABI and host-side evaluator of libcryptotl: parameter tables, keys, model banks, and the
// launch sequences of the encrypted dense layer (Eq. (1) of CryptoTL, Section 3.1), the x^2
// activation, replicate and rescale. Every arithmetic step runs in the HIP kernels; the host only
// samples client randomness, encodes FP64 slot vectors and orders launches on the caller's stream.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "ctl_internal.h"
#include "kernels.h"

using namespace ctl;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define CTL_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(CTL_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define CTL_TRY(expr)                  \
    do {                               \
        int rc_ = (expr);              \
        if (rc_ != CTL_OK) return rc_; \
    } while (0)

enum Family { F_NTT_FWD, F_NTT_INV, F_MODUP, F_KEYIP, F_DROP, F_MAC, F_ADD, F_TENSOR, F_INT_NTT, F_OTHER,
              F_MAC_FP, F_MAC_DIRECT, F_KEYIP_FP, F_NTT_FWD_FP, F_NTT_INV_FP, F_MODUP_FP, F_DROP_FP, F_COUNT };
// Names of the kernels each family brackets (k_mac and k_keyip: the MAC and the key product over
// integer primes, limb or 128-bit form; k_mac_fp and k_keyip_fp: over FP64 primes; k_mac_direct:
// the unstaged MAC of small batches, all primes in one launch; the transform families cover every
// prime of a launch, except that a looped launch runs one kernel per class and records its
// FP64-prime kernel under the _fp family).
const char *const kFamilyNames[F_COUNT] = {"k_ntt_fwd", "k_ntt_inv", "k_modup", "k_keyip", "k_drop",
                                            "k_mac", "k_add_terms", "k_tensor", "k_int_ntt", "other",
                                            "k_mac_fp", "k_mac_direct", "k_keyip_fp", "k_ntt_fwd_fp",
                                            "k_ntt_inv_fp", "k_modup_fp", "k_drop_fp"};

// Workspace slots: each grows on demand and is reused by later calls on the same context.
enum Slot {
    S_COEF, S_DIG, S_U, S_PLAST, S_ROT, S_INNER, S_SUM, S_LAST, S_TENSOR, S_SQ, S_REP,
    S_FWD_A, S_FWD_B, S_FWD_C, S_COEF2, S_ROT2, S_MISC, S_P_Z2, S_P_T, S_P_U, S_P_W, S_P_V, S_NTT_TMP, S_NTT_TMP2,
    S_COUNT
};

}  // namespace

struct ctl_ctx {
    HostParams hp;
    int device = 0;
    Tables tab{};
    void *tables_mem = nullptr;
    ctl_alloc_fn alloc = nullptr;
    ctl_free_fn free_fn = nullptr;
    void *user = nullptr;
    void *slot_ptr[S_COUNT] = {};
    size_t slot_bytes[S_COUNT] = {};
    std::unique_ptr<Encoder> enc;
    std::vector<PrimeConst> pc;
    bool ws_frozen = false;
    Knobs knobs;
    // the fixed scratch array of this context's GPU; while `arena` is set (inside the entry point
    // that allocates nothing) slot() carves buffers from it instead of the workspace
    u64 *scratch = nullptr;
    bool arena = false;
    size_t arena_used = 0;
    // lifetime: one reference for the context itself and one per live key or model handle made
    // on it; ctl_ctx_free drops the context's own (and releases the workspace at once), and the
    // tables and this struct go when the last reference does, whatever the order of the frees
    std::atomic<int> refs{1};
    // launch instrumentation
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;      // pairs (start, stop)
    std::vector<int> prof_fam;            // family of each recorded pair
    std::vector<double> prof_work;        // algorithmic work of each recorded launch
    std::vector<double> prof_fp;          // the part of it on FP64 primes
    std::vector<double> prof_bytes;       // algorithmic HBM bytes of each recorded launch (0: not modelled)
    std::vector<int> prof_layer_v;        // call site of each record: layer of the model (-1: none)
    std::vector<const char *> prof_phase_v;   // and phase of the layer (static strings)
    size_t prof_used = 0;
    int prof_layer = -1;                  // the current call site
    const char *prof_phase = "";
};

struct ctl_sk {
    ctl_ctx *ctx;
    std::vector<int64_t> s;
    u64 *d_s = nullptr;          // [np][N] NTT form
};

struct ctl_pk {
    ctl_ctx *ctx;
    u64 *d_pk = nullptr;         // [2][nq][N]
};

struct ctl_evk {
    ctl_ctx *ctx;
    std::map<u64, u64 *> keys;   // Galois element (0 = relinearization) -> [nq][2][np][N]
};

struct LayerPlan {
    int n_in, n_out, t, t1, t2, k, act;
    bool lazy = false;
    bool qp = false;              // baby steps over Q*P: the bank carries a row mod P
    double pt_scale;
    int kind = CTL_LAYER_DENSE;
    int f = 0;                    // convolution / pooling size
    int in_off = 0;               // slot offset of a dense layer's input (f - 1 after a pool)
    int rep_before = 0;           // replicate with this width before the layer (0: none)
    int nb = 0;                   // plaintexts in the bank (t1 * t2)
    std::vector<long> rots1;      // baby rotations; bank entry j >= 1 multiplies rot_{rots1[j-1]}
    double act_scale_in = 0;      // scale at the activation's input
    double act_coef[4] = {0, 0, 0, 0};
};

struct ctl_model {
    ctl_ctx *ctx;
    std::vector<LayerPlan> layers;
    std::vector<u64 *> banks;     // [t][k][N] NTT form per layer
    std::vector<int32_t> rotations;
    int block = 0, items = 0, k_out = 0;
    double scale_in = 0, scale_out = 0;
};

namespace {

// ---------------------------------------------------------------- memory
void *dev_alloc(ctl_ctx *c, size_t bytes, hipStream_t st) {
    if (bytes == 0) bytes = 256;
    if (c->alloc) return c->alloc(bytes, st, c->user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void dev_free(ctl_ctx *c, void *p, hipStream_t st) {
    if (!p) return;
    if (c->free_fn) c->free_fn(p, st, c->user);
    else (void)hipFree(p);
}

// Handles made on a context keep it alive (see ctl_ctx::refs).
void ctx_retain(ctl_ctx *c) { c->refs.fetch_add(1); }
void ctx_release(ctl_ctx *c) {
    if (c->refs.fetch_sub(1) != 1) return;
    (void)hipSetDevice(c->device);
    (void)hipFree(c->tables_mem);
    delete c;
}

int slot(ctl_ctx *c, Slot s, size_t words, hipStream_t st, u64 **out) {
    if (c->arena) {                            // carve from the scratch array, 256-byte aligned
        const size_t w = (std::max<size_t>(words, 1) + 31) / 32 * 32;
        if (!c->scratch || c->arena_used + w > kScratchWords)
            return fail(CTL_ENOMEM, "the call needs more than the fixed scratch array holds");
        *out = c->scratch + c->arena_used;
        c->arena_used += w;
        return CTL_OK;
    }
    const size_t bytes = std::max<size_t>(words * 8, 256);
    if (c->slot_bytes[s] < bytes) {
        if (c->ws_frozen)
            return fail(CTL_ENOMEM, "workspace is frozen and this call needs " + std::to_string(bytes) +
                                        " bytes in a slot holding " + std::to_string(c->slot_bytes[s]));
        CTL_HIP(hipStreamSynchronize(st));
        dev_free(c, c->slot_ptr[s], st);
        c->slot_ptr[s] = nullptr;
        c->slot_bytes[s] = 0;
        void *p = dev_alloc(c, bytes, st);
        if (!p) return fail(CTL_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
        c->slot_ptr[s] = p;
        c->slot_bytes[s] = bytes;
    }
    *out = static_cast<u64 *>(c->slot_ptr[s]);
    return CTL_OK;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// Buffer for a launch of `count` residue transforms split over N/1024 workgroups each (the NTT
// launches take it when the launch has fewer transforms than the ntt_split knob), or null for the
// one-workgroup form: at or above the knob, inside the entry point that allocates nothing, or when
// a frozen workspace cannot hold it (the one-workgroup form gives the same residues).
u64 *split_buf(ctl_ctx *c, hipStream_t st, int count, Slot which = S_NTT_TMP) {
    if (count >= c->knobs.ntt_split || c->arena) return nullptr;
    const std::string err = g_err;
    u64 *t = nullptr;
    // sized for the largest launch that splits, so that one small warm-up run reserves it
    if (slot(c, which, (size_t)std::max(count, c->knobs.ntt_split - 1) * c->hp.n, st, &t) != CTL_OK) {
        g_err = err;                             // not an error of the call: fall back
        return nullptr;
    }
    return t;
}

// Buffers of a split chain: an inverse transform of count_i residues fused into the forward
// transforms of their count_i * per targets (see launch_modup_chain); false when the forward
// launch does not split.
bool split_chain(ctl_ctx *c, hipStream_t st, int count_i, int per, u64 **tmp_i, u64 **tmp_f) {
    *tmp_f = split_buf(c, st, count_i * per);
    *tmp_i = *tmp_f ? split_buf(c, st, count_i, S_NTT_TMP2) : nullptr;
    return *tmp_i != nullptr;
}

// Brackets one launch with events when the context's instrumentation is on.
class Prof {
  public:
    Prof(ctl_ctx *c, Family f, hipStream_t st, double work, double fp_share = 0.0, double bytes = 0.0)
        : c_(c), st_(st), idx_(SIZE_MAX) {
        if (!c->prof_on || c->arena) return;     // no event creation inside the no-allocation call
        if (c->prof_used * 2 + 2 > c->prof_ev.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
            c->prof_ev.push_back(a);
            c->prof_ev.push_back(b);
            c->prof_fam.push_back(0);
            c->prof_work.push_back(0.0);
            c->prof_fp.push_back(0.0);
            c->prof_bytes.push_back(0.0);
            c->prof_layer_v.push_back(-1);
            c->prof_phase_v.push_back("");
        }
        idx_ = c->prof_used++;
        c->prof_fam[idx_] = f;
        c->prof_work[idx_] = work;
        c->prof_fp[idx_] = work * fp_share;
        c->prof_bytes[idx_] = bytes;
        c->prof_layer_v[idx_] = c->prof_layer;
        c->prof_phase_v[idx_] = c->prof_phase;
        (void)hipEventRecord(c->prof_ev[2 * idx_], st_);
    }
    ~Prof() {
        if (idx_ != SIZE_MAX) (void)hipEventRecord(c_->prof_ev[2 * idx_ + 1], st_);
    }
  private:
    ctl_ctx *c_;
    hipStream_t st_;
    size_t idx_;
};
// Call site recorded with the launches inside its scope: the layer of the model (layer < -1
// keeps the current one) and the phase of the layer.
class Site {
  public:
    Site(ctl_ctx *c, int layer, const char *phase) : c_(c), layer_(c->prof_layer), phase_(c->prof_phase) {
        if (layer >= -1) c->prof_layer = layer;
        if (phase) c->prof_phase = phase;
    }
    ~Site() {
        c_->prof_layer = layer_;
        c_->prof_phase = phase_;
    }
  private:
    ctl_ctx *c_;
    int layer_;
    const char *phase_;
};
constexpr int kKeepLayer = -2;

#define CTL_PROF(fam, work, share) Prof prof_##__LINE__(c, fam, st, (double)(work), (share))
#define CTL_PROFB(fam, work, share, bytes) Prof prof_##__LINE__(c, fam, st, (double)(work), (share), (double)(bytes))

// Share of the residues of a list of prime indices that run on the FP64 path.
double fp_share(const ctl_ctx *c, const int *primes, int n) {
    if (n <= 0) return 0.0;
    int f = 0;
    for (int i = 0; i < n; ++i) f += c->pc[primes[i]].fp ? 1 : 0;
    return (double)f / n;
}

// ModUp transforms: for each digit j the targets are the other k - 1 primes and P.
double modup_share(const ctl_ctx *c, int k) {
    int f = 0, n = 0;
    for (int j = 0; j < k; ++j)
        for (int t = 0; t <= k; ++t) {
            if (t == j) continue;
            f += c->pc[t < k ? t : c->hp.nq].fp ? 1 : 0;
            ++n;
        }
    return n ? (double)f / n : 0.0;
}

// Share for "targets 0..k-1 plus optionally P".
double fp_share_range(const ctl_ctx *c, int k, bool with_p) {
    int pr[kMaxMods], n = 0;
    for (int i = 0; i < k; ++i) pr[n++] = i;
    if (with_p) pr[n++] = c->hp.nq;
    return fp_share(c, pr, n);
}

// One NTT-bearing launch, bracketed per kernel: a looped launch (classes != 0) runs one kernel per
// arithmetic class, the FP64-prime one recorded under fam_fp with its share of the work.
template <typename Launch>
void transforms(ctl_ctx *c, hipStream_t st, Family fam, Family fam_fp, double work, double share, int classes,
                Launch &&launch) {
    if (!classes) {
        CTL_PROF(fam, work, share);
        launch(-1);
        return;
    }
    if (classes & 1) {
        CTL_PROF(fam_fp, work * share, 1.0);
        launch(0);
    }
    if (classes & 2) {
        CTL_PROF(fam, work * (1.0 - share), 0.0);
        launch(1);
    }
}

// The plaintext-product MAC over `rows` residue rows (the last one mod P when ext), bracketed per
// kernel: the FP64-prime and integer-prime launches, or the one unstaged launch of a small batch.
void run_mac(ctl_ctx *c, hipStream_t st, const u64 *ct, long ct_sb, const u64 *rot, long rot_sb, const u64 *bank,
             u64 *inner, int B, int rows, bool ext, int t1, int t2) {
    const int logn = c->hp.logn, nq = c->hp.nq;
    const double per_row = 2.0 * B * t1 * t2 * c->hp.n;
    // per residue row: the ciphertext and its rotations read once, the bank once, the sums written
    const double row_bytes = 8.0 * c->hp.n * (2.0 * B * t1 + (double)t1 * t2 + 2.0 * B * t2);
    int fp_rows = 0;
    for (int r = 0; r < rows; ++r) fp_rows += c->tab.host_fp[(ext && r == rows - 1) ? nq : r] ? 1 : 0;
    const int ext_nq = ext ? nq : -1;
    if (B <= c->knobs.mac_direct_max) {
        CTL_PROFB(F_MAC_DIRECT, per_row * rows, (double)fp_rows / rows, row_bytes * rows);
        launch_mac(logn, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, ext_nq, t1, t2, c->tab, c->knobs, st, 0);
        return;
    }
    if (fp_rows) {
        CTL_PROFB(F_MAC_FP, per_row * fp_rows, 1.0, row_bytes * fp_rows);
        launch_mac(logn, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, ext_nq, t1, t2, c->tab, c->knobs, st, 1);
    }
    if (fp_rows < rows) {
        CTL_PROFB(F_MAC, per_row * (rows - fp_rows), 0.0, row_bytes * (rows - fp_rows));
        launch_mac(logn, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, ext_nq, t1, t2, c->tab, c->knobs, st, 2);
    }
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(CTL_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return CTL_OK;
}

ResMap dense_map(int per, int prime_base = 0) {
    ResMap m{};
    m.per = per;
    m.ngrp = 1;
    m.off = 0;
    m.gstride = per;
    m.ostride = per;
    for (int i = 0; i < per; ++i) m.prime[i] = prime_base + i;
    return m;
}

// Handles made on one context may be used with any context of identical parameters on the same
// device (for example several contexts serving one parameter set on different streams).
bool same_params(const ctl_ctx *a, const ctl_ctx *b) {
    if (a == b) return true;
    if (a->device != b->device || a->hp.logn != b->hp.logn || a->hp.nq != b->hp.nq || a->hp.np != b->hp.np)
        return false;
    for (int i = 0; i < a->hp.np; ++i)
        if (a->hp.mods[i] != b->hp.mods[i]) return false;
    return true;
}

#define CTL_SAME(ctx, h, what)                                                                          \
    do {                                                                                                \
        if (!same_params((ctx), (h)->ctx))                                                              \
            return fail(CTL_EINVAL, what " was made for a context with other parameters or device");     \
    } while (0)

const u64 *find_key(const ctl_evk *evk, u64 g) {
    auto it = evk->keys.find(g);
    return it == evk->keys.end() ? nullptr : it->second;
}

// The evaluation keys of a batch: runs of consecutive ciphertexts that share one key set (one
// client). Key products run per run; every other kernel covers the whole batch.
struct KeySet {
    struct Run {
        const ctl_evk *evk;
        int b0, nb;
    };
    std::vector<Run> runs;
    KeySet slice(int b0, int nb) const;
};

// The key sets of ciphertexts b0 .. b0 + nb - 1, renumbered from 0.
KeySet KeySet::slice(int b0, int nb) const {
    KeySet out;
    for (const Run &r : runs) {
        const int lo = std::max(r.b0, b0), hi = std::min(r.b0 + r.nb, b0 + nb);
        if (lo < hi) out.runs.push_back({r.evk, lo - b0, hi - lo});
    }
    return out;
}

KeySet one_key_set(const ctl_evk *evk, int B) {
    KeySet ks;
    ks.runs.push_back({evk, 0, B});
    return ks;
}

// Every run holds key `id` (a Galois element, or 0 for the relinearization key); `what` names it.
int need_key(const KeySet &ks, u64 id, const std::string &what) {
    for (const KeySet::Run &r : ks.runs)
        if (!find_key(r.evk, id)) return fail(CTL_EKEY, "missing " + what);
    return CTL_OK;
}

// ---------------------------------------------------------------- building blocks
// ModUp of G polynomials d (k residues each, located by dmap, NTT form): iNTT, then the centered
// lift of each digit to the other primes and P and its NTT, into workspace slot S_DIG as
// [G][k][k+1][N] (*dig_out).
int modup_digits(ctl_ctx *c, hipStream_t st, int k, int G, const u64 *d, const ResMap &dmap, u64 **dig_out) {
    const int logn = c->hp.logn, nq = c->hp.nq;
    const long N = c->hp.n;
    u64 *coef, *dig;
    CTL_TRY(slot(c, S_DIG, (size_t)G * k * (k + 1) * N, st, &dig));
    u64 *ti, *tf;
    if (split_chain(c, st, G * k, k + 1, &ti, &tf)) {
        { CTL_PROF(F_NTT_INV, G * k, fp_share_range(c, k, false)); launch_modup_chain(logn, true, d, dmap, dig, G, k, nq, c->tab, st, ti, tf); }
        { CTL_PROF(F_MODUP, G * k * k, modup_share(c, k)); launch_modup_chain(logn, false, d, dmap, dig, G, k, nq, c->tab, st, ti, tf); }
        *dig_out = dig;
        return check_launch();
    }
    CTL_TRY(slot(c, S_COEF, (size_t)G * k * N, st, &coef));
    {
        u64 *sp = split_buf(c, st, G * k);
        transforms(c, st, F_NTT_INV, F_NTT_INV_FP, G * k, fp_share_range(c, k, false),
                   ntt_loop_classes(G * k, dmap, c->tab, c->knobs, sp), [&](int cls) {
                       launch_ntt(logn, true, d, dmap, coef, dense_map(k), G * k, c->tab, c->knobs, st, sp, cls);
                   });
    }
    {
        u64 *sp = split_buf(c, st, G * k * (k + 1));
        transforms(c, st, F_MODUP, F_MODUP_FP, G * k * k, modup_share(c, k),
                   modup_loop_classes(G, k, nq, c->tab, c->knobs, sp), [&](int cls) {
                       launch_modup(logn, coef, d, dmap, dig, G, k, nq, c->tab, c->knobs, st, sp, cls);
                   });
    }
    *dig_out = dig;
    return check_launch();
}

// Key products of B ciphertexts and R rotations from ModUp digits (ciphertext b at dig + b db;
// hoisted: the same digits for every rotation, else rotation r's at + r k(k+1)N): U[b][r] =
// sum_j digit_j * key_r[j] gathered through sigma_{gal[r]} (+ the fold term), [2][k+1][N] at
// U + b U_sb + r 2(k+1)N. One launch per key set.
int key_product(ctl_ctx *c, hipStream_t st, int k, int B, int R, const u64 *dig, long db, bool hoisted,
                const KeySet &ks, const u64 *key_ids, const u64 *gal, const KeyFold *fold, u64 *U, long U_sb) {
    const int logn = c->hp.logn, nq = c->hp.nq;
    const long N = c->hp.n;
    if (R > kMaxKeysPerLaunch) return fail(CTL_EINVAL, "too many rotations in one layer");
    const long dsz = (long)k * (k + 1) * N;
    KeyFold fd{};
    if (fold) fd = *fold;
    auto key_list = [&](const KeySet::Run &run, KeyList &kl) {
        kl = KeyList{};
        for (int r = 0; r < R; ++r) {
            kl.key[r] = find_key(run.evk, key_ids[r]);
            if (!kl.key[r]) return false;
            kl.gal[r] = gal[r];
            kl.ginv[r] = galois_inv(logn, gal[r]);
        }
        return true;
    };
    KeyList kl;
    for (const KeySet::Run &run : ks.runs)          // every key present before anything is launched
        if (!key_list(run, kl)) return fail(CTL_EKEY, "missing evaluation key");
    RowSet rows[KIP_CLASSES];
    keyip_rows(k, nq, c->tab, c->knobs, rows);
    for (int cls = 0; cls < KIP_CLASSES; ++cls) {  // one launch per arithmetic class and key set
        const RowSet &rs = rows[cls];
        if (rs.n == 0) continue;
        int fold_rows = 0;
        for (int i = 0; i < rs.n; ++i) fold_rows += fold && fold->src && rs.t[i] < fold->rows ? 1 : 0;
        // algorithmic bytes of these rows: digits (once per ciphertext when hoisted), each key
        // set's keys, the outputs, and the fold term's words
        const double kip_bytes = 8.0 * N * ((double)B * (hoisted ? 1 : R) * k * rs.n +
                                            (double)ks.runs.size() * R * 2 * k * rs.n + (double)B * R * 2 * rs.n +
                                            (fold && fold->src ? (double)B * (fold->sr ? R : 1) * fold_rows : 0.0));
        CTL_PROFB(cls == KIP_FP ? F_KEYIP_FP : F_KEYIP, 2.0 * B * R * rs.n * k * N, cls == KIP_FP ? 1.0 : 0.0,
                  kip_bytes);
        for (const KeySet::Run &run : ks.runs) {
            key_list(run, kl);
            KeyFold fr = fd;
            if (fr.src) fr.src += run.b0 * fr.sb;
            launch_keyip(logn, k, cls, rs, dig + run.b0 * db, db, hoisted ? 0 : dsz, kl, R, U + run.b0 * U_sb,
                         U_sb, fr, run.nb, nq, c->tab, c->knobs, st);
        }
    }
    return check_launch();
}

// Raise and multiply: for G = B R polynomials d (k residues each, located by dmap over B*R*k
// residues, group order (b, r)), U[b][r] = sum_j ModUp(d)_j * key_r[j] gathered through
// sigma_{gal[r]} (plus the fold term, see KeyFold), as [2][k+1][N] over q_0..q_{k-1}, P.
// `hoisted` = the same d for every r (dmap covers B*k residues only). U goes to U_dst with batch
// stride U_sb and [R][2][k+1][N] per ciphertext, or, with U_dst null, to workspace slot S_U as
// [B][R][2][k+1][N]; *U_out receives its address.
int keyswitch_raise(ctl_ctx *c, hipStream_t st, int k, int B, int R, const u64 *d, const ResMap &dmap,
                    bool hoisted, const KeySet &ks, const u64 *key_ids, const u64 *gal, u64 **U_out,
                    const KeyFold *fold = nullptr, u64 *U_dst = nullptr, long U_sb = 0) {
    const long N = c->hp.n;
    if (R > kMaxKeysPerLaunch) return fail(CTL_EINVAL, "too many rotations in one layer");
    const int G = hoisted ? B : B * R;
    u64 *dig, *U;
    if (U_dst) {
        U = U_dst;
    } else {
        CTL_TRY(slot(c, S_U, (size_t)B * R * 2 * (k + 1) * N, st, &U));
        U_sb = (long)R * 2 * (k + 1) * N;
    }
    CTL_TRY(modup_digits(c, st, k, G, d, dmap, &dig));
    const long dsz = (long)k * (k + 1) * N, db = hoisted ? dsz : (long)R * dsz;
    CTL_TRY(key_product(c, st, k, B, R, dig, db, hoisted, ks, key_ids, gal, fold, U, U_sb));
    *U_out = U;
    return CTL_OK;
}

// Lower G2 = 2 B R extended polynomials U ([G2][k+1][N]) by ModDown into out ([G2][k][N]),
// adding `add` (see DropAdd).
int keyswitch_lower(ctl_ctx *c, hipStream_t st, int k, int groups, const u64 *U, const DropAdd &add, u64 *out) {
    const int logn = c->hp.logn, nq = c->hp.nq;
    const long N = c->hp.n;
    ResMap pm{};
    pm.per = 1;
    pm.ngrp = 1;
    pm.off = k;
    pm.gstride = k + 1;
    pm.ostride = k + 1;
    pm.prime[0] = nq;
    u64 *ti, *tf;
    if (split_chain(c, st, groups, k, &ti, &tf)) {
        const GrpMap xm{0, (k + 1) * N, 0, 1};
        { CTL_PROF(F_NTT_INV, groups, fp_share_range(c, 0, true)); launch_drop_chain(logn, true, U, pm, U, xm, out, groups, k, nq, add, c->tab, st, ti, tf); }
        { CTL_PROF(F_DROP, (double)groups * k, fp_share_range(c, k, false)); launch_drop_chain(logn, false, U, pm, U, xm, out, groups, k, nq, add, c->tab, st, ti, tf); }
        return check_launch();
    }
    u64 *plast;                                  // coefficients of the P rows (not in the chain)
    CTL_TRY(slot(c, S_PLAST, (size_t)groups * N, st, &plast));
    {
        u64 *sp = split_buf(c, st, groups);
        transforms(c, st, F_NTT_INV, F_NTT_INV_FP, groups, fp_share_range(c, 0, true),
                   ntt_loop_classes(groups, pm, c->tab, c->knobs, sp), [&](int cls) {
                       launch_ntt(logn, true, U, pm, plast, dense_map(1, nq), groups, c->tab, c->knobs, st, sp, cls);
                   });
    }
    {
        u64 *sp = split_buf(c, st, groups * k);
        transforms(c, st, F_DROP, F_DROP_FP, (double)groups * k, fp_share_range(c, k, false),
                   drop_loop_classes(groups, k, c->tab, c->knobs, sp), [&](int cls) {
                       launch_drop(logn, U, plast, out, groups, k, nq, add, c->tab, c->knobs, st, nullptr, sp, cls);
                   });
    }
    return check_launch();
}

// Full key switch: out[b][r] = (KS0 + addend, KS1) as [B][R][2][k][N].
int keyswitch_batch(ctl_ctx *c, hipStream_t st, int k, int B, int R, const u64 *d, const ResMap &dmap,
                    bool hoisted, const KeySet &ks, const u64 *key_ids, const u64 *gal, const DropAdd &add,
                    u64 *out) {
    u64 *U;
    CTL_TRY(keyswitch_raise(c, st, k, B, R, d, dmap, hoisted, ks, key_ids, gal, &U));
    return keyswitch_lower(c, st, k, B * R * 2, U, add, out);
}

// Rescale [B][2][k][N] -> [B][2][k-1][N].
int rescale_batch(ctl_ctx *c, hipStream_t st, int k, int B, const u64 *in, u64 *out) {
    const int logn = c->hp.logn;
    const long N = c->hp.n;
    if (k < 2) return fail(CTL_ELEVEL, "cannot rescale at one prime");
    ResMap m{};
    m.per = 1;
    m.ngrp = 1;
    m.off = k - 1;
    m.gstride = k;
    m.ostride = k;
    m.prime[0] = k - 1;
    u64 *ti, *tf;
    if (split_chain(c, st, B * 2, k - 1, &ti, &tf)) {
        DropAdd add{};
        add.R = 1;
        add.mask = 0;
        add.gal[0] = 1;
        const GrpMap xm{0, k * N, 0, 1};
        { CTL_PROF(F_NTT_INV, B * 2, fp_share(c, &m.prime[0], 1)); launch_drop_chain(logn, true, in, m, in, xm, out, B * 2, k - 1, k - 1, add, c->tab, st, ti, tf); }
        { CTL_PROF(F_DROP, B * 2 * (k - 1), fp_share_range(c, k - 1, false)); launch_drop_chain(logn, false, in, m, in, xm, out, B * 2, k - 1, k - 1, add, c->tab, st, ti, tf); }
        return check_launch();
    }
    u64 *last;                                   // coefficients of the dropped prime (not in the chain)
    CTL_TRY(slot(c, S_LAST, (size_t)B * 2 * N, st, &last));
    {
        u64 *sp = split_buf(c, st, B * 2);
        transforms(c, st, F_NTT_INV, F_NTT_INV_FP, B * 2, fp_share(c, &m.prime[0], 1),
                   ntt_loop_classes(B * 2, m, c->tab, c->knobs, sp), [&](int cls) {
                       launch_ntt(logn, true, in, m, last, dense_map(1, k - 1), B * 2, c->tab, c->knobs, st, sp, cls);
                   });
    }
    DropAdd add{};
    add.R = 1;
    add.mask = 0;
    add.gal[0] = 1;
    {
        u64 *sp = split_buf(c, st, B * 2 * (k - 1));
        transforms(c, st, F_DROP, F_DROP_FP, B * 2 * (k - 1), fp_share_range(c, k - 1, false),
                   drop_loop_classes(B * 2, k - 1, c->tab, c->knobs, sp), [&](int cls) {
                       launch_drop(logn, in, last, out, B * 2, k - 1, k - 1, add, c->tab, c->knobs, st, nullptr, sp, cls);
                   });
    }
    return check_launch();
}

// ModDown of G = 2 B extended polynomials U ([G][k+1][N]) by P, adding `add` (R = 1, no rotation),
// then the rescale by q_{k-1}, into out ([B][2][k-1][N]). With the fuse_rescale knob set both run as
// one pass (launch_drop_rescale: the inverse transforms of rows k - 1 and P, then k - 1 forward
// transforms per polynomial, the residues of the two steps; U's row k - 1 takes the addend's
// first; a split chain for few polynomials); otherwise ModDown into mid ([B][2][k][N]) and the
// rescale after it.
int lower_rescale(ctl_ctx *c, hipStream_t st, int k, int B, u64 *U, const DropAdd &add, u64 *mid, u64 *out) {
    if (k < 2) return fail(CTL_ELEVEL, "cannot rescale at one prime");
    if (!c->knobs.fuse_rescale || (add.mask && (add.R != 1 || add.gal[0] != 1))) {
        if (!mid) return fail(CTL_EINVAL, "ModDown apart from the rescale needs an intermediate buffer");
        CTL_TRY(keyswitch_lower(c, st, k, B * 2, U, add, mid));
        return rescale_batch(c, st, k, B, mid, out);
    }
    const int logn = c->hp.logn, nq = c->hp.nq, kl = k - 1, G = B * 2;
    const long N = c->hp.n, xs = (long)(k + 1) * N;
    if (add.mask) { CTL_PROF(F_ADD, (double)G * N, 0.0); launch_fold_last(logn, U, xs, G, kl, nq, add, c->tab, st); }
    {
        u64 *tf = split_buf(c, st, G * kl), *ti = tf ? split_buf(c, st, G * 2, S_NTT_TMP2) : nullptr;
        if (ti) {
            const int pr[2] = {kl, nq};
            { CTL_PROF(F_NTT_INV, G * 2, fp_share(c, pr, 2)); launch_drop_rescale_chain(logn, true, U, xs, out, G, kl, nq, add, c->tab, st, ti, tf); }
            { CTL_PROF(F_DROP, (double)G * kl, fp_share_range(c, kl, false)); launch_drop_rescale_chain(logn, false, U, xs, out, G, kl, nq, add, c->tab, st, ti, tf); }
            return check_launch();
        }
    }
    u64 *coef;
    CTL_TRY(slot(c, S_PLAST, (size_t)G * 2 * N, st, &coef));
    ResMap im{};                              // rows k - 1 and P of each polynomial
    im.per = 2;
    im.ngrp = 1;
    im.off = kl;
    im.gstride = k + 1;
    im.ostride = k + 1;
    im.prime[0] = kl;
    im.prime[1] = nq;
    {
        u64 *sp = split_buf(c, st, G * 2);
        transforms(c, st, F_NTT_INV, F_NTT_INV_FP, G * 2, fp_share(c, im.prime, 2),
                   ntt_loop_classes(G * 2, im, c->tab, c->knobs, sp), [&](int cls) {
                       launch_ntt(logn, true, U, im, coef, dense_map(2), G * 2, c->tab, c->knobs, st, sp, cls);
                   });
    }
    {
        u64 *sp = split_buf(c, st, G * kl);
        transforms(c, st, F_DROP, F_DROP_FP, (double)G * kl, fp_share_range(c, kl, false),
                   drop_loop_classes(G, kl, c->tab, c->knobs, sp), [&](int cls) {
                       launch_drop_rescale(logn, U, xs, coef, out, G, kl, nq, add, c->tab, c->knobs, st, sp, cls);
                   });
    }
    return check_launch();
}

ResMap c1_map(int k) {        // the c1 residues of a [B][2][k][N] batch
    ResMap m{};
    m.per = k;
    m.ngrp = 1;
    m.off = k;
    m.gstride = 2 * k;
    m.ostride = 2 * k;
    for (int i = 0; i < k; ++i) m.prime[i] = i;
    return m;
}

int rotate_batch(ctl_ctx *c, hipStream_t st, const KeySet &ks, int k, int B, long rot, const u64 *in, u64 *out) {
    const u64 g = galois_elt(c->hp.logn, rot);
    const long N = c->hp.n;
    if (g == 1) {
        CTL_HIP(hipMemcpyAsync(out, in, (size_t)B * 2 * k * N * 8, hipMemcpyDeviceToDevice, st));
        return CTL_OK;
    }
    CTL_TRY(need_key(ks, g, "Galois key for rotation " + std::to_string(rot)));
    DropAdd add{};
    add.base = in;
    add.sb = 2L * k * N;
    add.R = 1;
    add.mask = 1;
    add.gal[0] = g;
    return keyswitch_batch(c, st, k, B, 1, in, c1_map(k), false, ks, &g, &g, add, out);
}

int replicate_batch(ctl_ctx *c, hipStream_t st, const KeySet &ks, int k, int B, int width, const u64 *in, u64 *out) {
    const long N = c->hp.n;
    u64 *rot;
    CTL_TRY(slot(c, S_REP, (size_t)B * 2 * k * N, st, &rot));
    CTL_TRY(rotate_batch(c, st, ks, k, B, -(long)width, in, rot));
    { CTL_PROF(F_ADD, 2.0 * B * k * N, 0.0); launch_add_terms(c->hp.logn, in, 2L * k * N, rot, 2L * k * N, 0, 1, out, B, k, c->tab, st); }
    return check_launch();
}

// a x b: tensor, relinearization, rescale ([B][2][k][N] each -> [B][2][k-1][N]); a == b squares.
int mul_batch(ctl_ctx *c, hipStream_t st, const KeySet &ks, int k, int B, const u64 *a, const u64 *b, u64 *out) {
    const long N = c->hp.n;
    CTL_TRY(need_key(ks, 0, "relinearization key"));
    if (k < 2) return fail(CTL_ELEVEL, "a ciphertext product needs at least two primes");
    u64 *t3, *sq = nullptr;
    CTL_TRY(slot(c, S_TENSOR, (size_t)B * 3 * k * N, st, &t3));
    if (!c->knobs.fuse_rescale) CTL_TRY(slot(c, S_SQ, (size_t)B * 2 * k * N, st, &sq));
    { CTL_PROF(F_TENSOR, 4.0 * B * k * N, 0.0); launch_tensor(c->hp.logn, a, b, t3, B, k, c->tab, st); }
    ResMap dm{};
    dm.per = k;
    dm.ngrp = 1;
    dm.off = 2 * k;
    dm.gstride = 3 * k;
    dm.ostride = 3 * k;
    for (int i = 0; i < k; ++i) dm.prime[i] = i;
    DropAdd add{};
    add.base = t3;
    add.sb = 3L * k * N;
    add.sc = (long)k * N;
    add.R = 1;
    add.mask = 3;
    add.gal[0] = 1;
    const u64 rlk_id = 0, one = 1;
    u64 *U;
    CTL_TRY(keyswitch_raise(c, st, k, B, 1, t3, dm, false, ks, &rlk_id, &one, &U));
    return lower_rescale(c, st, k, B, U, add, sq, out);
}

int square_batch(ctl_ctx *c, hipStream_t st, const KeySet &ks, int k, int B, const u64 *in, u64 *out) {
    return mul_batch(c, st, ks, k, B, in, in, out);
}

u64 signed_mod(int64_t v, u64 q) {
    const u64 m = (u64)(v < 0 ? -(v + 1) : v) % q;      // |v| - 1 for negatives (no overflow at INT64_MIN)
    if (v >= 0) return m;
    const u64 a = (m + 1) % q;
    return a ? q - a : 0;
}

// out = in * mul + add (add to c0), keeping the first k_out of k_in residues per polynomial.
int affine_batch(ctl_ctx *c, hipStream_t st, int B, int k_in, int k_out, const u64 *in, int64_t mul, int64_t add,
                 u64 *out) {
    AffineConst ac{};
    for (int i = 0; i < k_out; ++i) {
        const u64 q = c->hp.mods[i];
        ac.mul[i] = signed_mod(mul, q);
        ac.muls[i] = (u64)(((u128)ac.mul[i] << 64) / q);
        ac.add[i] = signed_mod(add, q);
    }
    { CTL_PROF(F_ADD, 2.0 * B * k_out * c->hp.n, 0.0); launch_affine(c->hp.logn, in, out, B, k_in, k_out, ac, c->tab, st); }
    return check_launch();
}

// Integer constants of the degree-3 activation at k primes and input scale S (see ctl_poly3).
double poly3_consts(const ctl_ctx *c, int k, double S, const double *coef, int64_t *C) {
    const double qa = (double)c->hp.mods[k - 1], qb = (double)c->hp.mods[k - 2];
    const double S2 = (S * S) / qa;
    const double S3 = (S2 * S2) / qb;
    C[3] = std::llround(coef[3] * S);
    C[2] = std::llround(coef[2] * S2);
    C[1] = std::llround(coef[1] * ((S3 * qa) / S));
    C[0] = std::llround(coef[0] * S3);
    return S3;
}

bool poly3_consts_ok(const ctl_ctx *c, int k, double S, const double *coef) {
    const double qa = (double)c->hp.mods[k - 1], qb = (double)c->hp.mods[k - 2];
    const double S2 = (S * S) / qa, S3 = (S2 * S2) / qb;
    const double v[4] = {coef[0] * S3, coef[1] * ((S3 * qa) / S), coef[2] * S2, coef[3] * S};
    for (double x : v)
        if (!std::isfinite(x) || std::fabs(x) >= 4611686018427387904.0) return false;
    return true;
}

// c0 + c1 z + c2 z^2 + c3 z^3 on [B][2][k][N] -> [B][2][k-2][N] (schedule in ctl.h).
int poly3_batch(ctl_ctx *c, hipStream_t st, const KeySet &ks, int k, int B, double S, const double *coef,
                const u64 *in, u64 *out) {
    if (k < 3) return fail(CTL_ELEVEL, "the cubic activation needs at least three primes");
    if (!poly3_consts_ok(c, k, S, coef)) return fail(CTL_ESCALE, "activation constant out of range");
    const long N = c->hp.n;
    int64_t C[4];
    poly3_consts(c, k, S, coef, C);
    u64 *z2, *t, *u, *w, *v;
    CTL_TRY(slot(c, S_P_Z2, (size_t)B * 2 * (k - 1) * N, st, &z2));
    CTL_TRY(slot(c, S_P_T, (size_t)B * 2 * k * N, st, &t));
    CTL_TRY(slot(c, S_P_U, (size_t)B * 2 * (k - 1) * N, st, &u));
    CTL_TRY(slot(c, S_P_W, (size_t)B * 2 * (k - 2) * N, st, &w));
    CTL_TRY(slot(c, S_P_V, (size_t)B * 2 * (k - 2) * N, st, &v));
    CTL_TRY(square_batch(c, st, ks, k, B, in, z2));
    CTL_TRY(affine_batch(c, st, B, k, k, in, C[3], 0, t));
    CTL_TRY(rescale_batch(c, st, k, B, t, u));
    CTL_TRY(affine_batch(c, st, B, k - 1, k - 1, u, 1, C[2], u));
    CTL_TRY(mul_batch(c, st, ks, k - 1, B, z2, u, w));
    CTL_TRY(affine_batch(c, st, B, k, k, in, C[1], 0, t));
    CTL_TRY(rescale_batch(c, st, k, B, t, u));
    CTL_TRY(affine_batch(c, st, B, k - 1, k - 2, u, 1, C[0], v));
    { CTL_PROF(F_ADD, 2.0 * B * (k - 2) * N, 0.0); launch_add_terms(c->hp.logn, w, 2L * (k - 2) * N, v, 2L * (k - 2) * N, 0, 1, out, B, k - 2, c->tab, st); }
    return check_launch();
}

// Dense layer with the baby steps kept over Q*P (double hoisting, see CTL_LAYER_BABY_QP), for a
// batch grouped by model: group g is counts[g] consecutive ciphertexts evaluated by layer li of
// models[g] (every one a layer with baby steps over Q*P at the same input level k). Per group,
// with rot~ etc. over its own ciphertexts:
//   rot~[b][0] = P ct,  rot~[b][j] = U_j + (P sigma_j(c0), 0)        [B][t1][2][k+1][N]
//   inner~[b][k2] = sum_j pt~_{k2 t1 + j} rot~[b][j]                   [B][t2][2][k+1][N]
//   I1[b][k2-1] = ModDown(c1 of inner~[b][k2]), k2 >= 1                [B][t2-1][k][N]
//   usum[b] = inner~[b][0] + sum_{k2 >= 1} (KS_k2(sigma I1) + (sigma(c0 of inner~[b][k2]), 0))
//   out = rescale(ModDown(usum)).
// The hoisted ModUp of every c1, the ModUp of every I1, the final ModDown and the rescale each run
// once over the whole batch; key products, MACs and giant-step sums run per group. The bank of
// such a layer carries a last row mod P ([t][k+1][N]).
struct QpGroup {
    const ctl_model *m;
    int B, b0;                        // ciphertexts and the first one
    int t1, t2, R1, R2;
    std::vector<u64> gal1, gal2;
    long rot_off, inner_off, i1_off;  // words into the shared buffers
};

int dense_qp_groups(ctl_ctx *c, hipStream_t st, const ctl_model *const *models, const int *counts, int G, int li,
                    const KeySet &ks, const u64 *in, u64 *out) {
    const int logn = c->hp.logn, nq = c->hp.nq, k = models[0]->layers[li].k;
    const long N = c->hp.n, ctw = 2L * k * N, ext = 2L * (k + 1) * N, dsz = (long)k * (k + 1) * N;
    std::vector<QpGroup> gs(G);
    int B = 0;
    long rot_w = 0, inner_w = 0, i1_w = 0;
    for (int g = 0; g < G; ++g) {
        const LayerPlan &L = models[g]->layers[li];
        QpGroup &q = gs[g];
        q.m = models[g];
        q.B = counts[g];
        q.b0 = B;
        q.t1 = L.t1;
        q.t2 = L.t2;
        q.R1 = L.t1 - 1;
        q.R2 = L.t2 - 1;
        for (int j = 1; j < L.t1; ++j) q.gal1.push_back(galois_elt(logn, L.rots1[j - 1]));
        for (int k2 = 1; k2 < L.t2; ++k2) q.gal2.push_back(galois_elt(logn, (long)k2 * L.t1));
        q.rot_off = rot_w;
        q.inner_off = inner_w;
        q.i1_off = i1_w;
        rot_w += (long)q.B * q.t1 * ext;
        inner_w += q.t2 > 1 ? (long)q.B * q.t2 * ext : 0;      // t2 = 1: the MAC writes the sum
        i1_w += (long)q.B * q.R2;
        B += q.B;
    }
    u64 *rot, *inner = nullptr, *usum, *acc;
    CTL_TRY(slot(c, S_ROT, (size_t)rot_w, st, &rot));
    if (inner_w) CTL_TRY(slot(c, S_INNER, (size_t)inner_w, st, &inner));
    CTL_TRY(slot(c, S_ROT2, (size_t)B * ext, st, &usum));
    CTL_TRY(slot(c, S_SUM, (size_t)B * ctw, st, &acc));
    {
        Site site(c, kKeepLayer, "baby steps");
        for (const QpGroup &q : gs) {
            CTL_PROF(F_ADD, (double)q.B * ext, 0.0);
            launch_times_p(logn, in + q.b0 * ctw, rot + q.rot_off, (long)q.t1 * ext, q.B, k, nq, c->tab, st);
        }
        bool any_baby = false;
        for (const QpGroup &q : gs) any_baby = any_baby || q.R1 > 0;
        if (any_baby) {
            u64 *dig;
            CTL_TRY(modup_digits(c, st, k, B, in, c1_map(k), &dig));       // one ModUp for every group
            for (const QpGroup &q : gs) {
                if (q.R1 <= 0) continue;
                KeyFold fd{};
                fd.src = in + q.b0 * ctw;           // c0, gathered through sigma_j and scaled by P
                fd.sb = ctw;
                fd.sr = 0;
                fd.rows = k;
                for (int t = 0; t < k; ++t) fd.mul[t] = c->hp.mods[nq] % c->hp.mods[t];
                CTL_TRY(key_product(c, st, k, q.B, q.R1, dig + q.b0 * dsz, dsz, true, ks.slice(q.b0, q.B),
                                    q.gal1.data(), q.gal1.data(), &fd, rot + q.rot_off + ext, (long)q.t1 * ext));
            }
        }
    }
    {
        Site site(c, kKeepLayer, "mac");
        for (const QpGroup &q : gs) {
            u64 *dst = q.t2 > 1 ? inner + q.inner_off : usum + q.b0 * ext;
            const u64 *r0 = rot + q.rot_off;
            run_mac(c, st, r0, (long)q.t1 * ext, r0 + ext, (long)q.t1 * ext, q.m->banks[li], dst, q.B, k + 1, true,
                    q.t1, q.t2);
        }
        CTL_TRY(check_launch());
    }
    if (i1_w > 0) {
        Site site(c, kKeepLayer, "giant steps");
        DropAdd none{};
        none.R = 1;
        none.mask = 0;
        none.gal[0] = 1;
        u64 *i1, *plast;
        CTL_TRY(slot(c, S_COEF2, (size_t)i1_w * k * N, st, &i1));
        CTL_TRY(slot(c, S_PLAST, (size_t)i1_w * N, st, &plast));
        for (const QpGroup &q : gs) {              // I1 = ModDown of c1 of inner~[b][k2], k2 >= 1
            if (q.R2 <= 0) continue;
            const u64 *ig = inner + q.inner_off;
            ResMap pm{};                            // the P rows of those c1
            pm.per = 1;
            pm.ngrp = q.R2;
            pm.off = 3L * (k + 1) + k;
            pm.gstride = 2L * (k + 1);
            pm.ostride = (long)q.t2 * 2 * (k + 1);
            pm.prime[0] = nq;
            GrpMap xm{3L * (k + 1) * N, (long)q.t2 * ext, ext, q.R2};
            u64 *ti, *tf;
            if (split_chain(c, st, q.B * q.R2, k, &ti, &tf)) {
                u64 *o = i1 + q.i1_off * k * N;
                { CTL_PROF(F_NTT_INV, q.B * q.R2, fp_share_range(c, 0, true)); launch_drop_chain(logn, true, ig, pm, ig, xm, o, q.B * q.R2, k, nq, none, c->tab, st, ti, tf); }
                { CTL_PROF(F_DROP, (double)q.B * q.R2 * k, fp_share_range(c, k, false)); launch_drop_chain(logn, false, ig, pm, ig, xm, o, q.B * q.R2, k, nq, none, c->tab, st, ti, tf); }
                continue;
            }
            {
                u64 *sp = split_buf(c, st, q.B * q.R2);
                transforms(c, st, F_NTT_INV, F_NTT_INV_FP, q.B * q.R2, fp_share_range(c, 0, true),
                           ntt_loop_classes(q.B * q.R2, pm, c->tab, c->knobs, sp), [&](int cls) {
                               launch_ntt(logn, true, ig, pm, plast + q.i1_off * N, dense_map(1, nq), q.B * q.R2, c->tab,
                                          c->knobs, st, sp, cls);
                           });
            }
            {
                u64 *sp = split_buf(c, st, q.B * q.R2 * k);
                transforms(c, st, F_DROP, F_DROP_FP, (double)q.B * q.R2 * k, fp_share_range(c, k, false),
                           drop_loop_classes(q.B * q.R2, k, c->tab, c->knobs, sp), [&](int cls) {
                               launch_drop(logn, ig, plast + q.i1_off * N, i1 + q.i1_off * k * N, q.B * q.R2, k, nq, none,
                                           c->tab, c->knobs, st, &xm, sp, cls);
                           });
            }
        }
        u64 *dig, *U;
        CTL_TRY(modup_digits(c, st, k, (int)i1_w, i1, dense_map(k), &dig));   // one ModUp for every group
        CTL_TRY(slot(c, S_U, (size_t)i1_w * ext, st, &U));
        GalList one{};
        for (int r = 0; r < kMaxKeysPerLaunch; ++r) one.g[r] = 1;
        for (const QpGroup &q : gs) {
            if (q.R2 <= 0) continue;
            const u64 *ig = inner + q.inner_off;
            KeyFold fg{};
            fg.src = ig + ext;                      // c0 of inner~[b][1], all k + 1 rows
            fg.sb = (long)q.t2 * ext;
            fg.sr = ext;
            fg.rows = k + 1;
            for (int t = 0; t <= k; ++t) fg.mul[t] = 1;
            u64 *Ug = U + q.i1_off * ext;
            CTL_TRY(key_product(c, st, k, q.B, q.R2, dig + q.i1_off * dsz, (long)q.R2 * dsz, false,
                                ks.slice(q.b0, q.B), q.gal2.data(), q.gal2.data(), &fg, Ug, (long)q.R2 * ext));
            { CTL_PROF(F_ADD, (double)q.B * ext, 0.0); launch_sum_gather(logn, usum + q.b0 * ext, ext, ig, (long)q.t2 * ext, Ug, (long)q.R2 * ext, ext, q.R2, k + 1, true, 3, one, q.B, nq, c->tab, st); }
        }
        CTL_TRY(check_launch());
    }
    DropAdd none{};
    none.R = 1;
    none.mask = 0;
    none.gal[0] = 1;
    if (c->knobs.fuse_rescale) {
        Site s(c, kKeepLayer, "moddown + rescale");
        return lower_rescale(c, st, k, B, usum, none, acc, out);
    }
    { Site s(c, kKeepLayer, "moddown"); CTL_TRY(keyswitch_lower(c, st, k, B * 2, usum, none, acc)); }
    Site s(c, kKeepLayer, "rescale");
    return rescale_batch(c, st, k, B, acc, out);
}

int dense_batch(ctl_ctx *c, hipStream_t st, const ctl_model *m, int li, const KeySet &ks, int B,
                const u64 *in, u64 *out) {
    const LayerPlan &L = m->layers[li];
    const int logn = c->hp.logn, k = L.k, t1 = L.t1, t2 = L.t2;
    const long N = c->hp.n, ctw = 2L * k * N;
    const int R1 = t1 - 1, R2 = t2 - 1;
    if (R1 > kMaxKeysPerLaunch || R2 > kMaxKeysPerLaunch)
        return fail(CTL_EINVAL, "t1 and t2 must be at most 65");
    std::vector<u64> gal1(R1), gal2(R2);
    for (int j = 1; j < t1; ++j) {
        gal1[j - 1] = galois_elt(logn, L.rots1[j - 1]);
        CTL_TRY(need_key(ks, gal1[j - 1], "Galois key for rotation " + std::to_string(L.rots1[j - 1])));
    }
    for (int k2 = 1; k2 < t2; ++k2) {
        gal2[k2 - 1] = galois_elt(logn, (long)k2 * t1);
        CTL_TRY(need_key(ks, gal2[k2 - 1], "Galois key for rotation " + std::to_string(k2 * t1)));
    }
    if (L.qp) {
        const int cnt = B;
        return dense_qp_groups(c, st, &m, &cnt, 1, li, ks, in, out);
    }
    u64 *rot, *inner;
    CTL_TRY(slot(c, S_ROT, (size_t)B * std::max(R1, 1) * ctw, st, &rot));
    CTL_TRY(slot(c, S_INNER, (size_t)B * t2 * ctw, st, &inner));
    // baby steps rot_j(ct), j = 1..t1-1, sharing one ModUp of c1
    Site baby(c, kKeepLayer, "baby steps");
    if (R1 > 0) {
        DropAdd add{};
        add.base = in;
        add.sb = ctw;
        add.sr = 0;
        add.R = R1;
        add.mask = 1;
        for (int r = 0; r < R1; ++r) add.gal[r] = gal1[r];
        CTL_TRY(keyswitch_batch(c, st, k, B, R1, in, c1_map(k), true, ks, gal1.data(), gal1.data(), add, rot));
    }
    // inner_k2 = sum_j diag'_{k2 t1 + j} * rot_j(ct)
    { Site s(c, kKeepLayer, "mac"); run_mac(c, st, in, ctw, rot, (long)R1 * ctw, m->banks[li], inner, B, k, false, t1, t2); }
    CTL_TRY(check_launch());
    Site giant(c, kKeepLayer, "giant steps");
    const u64 *sum = inner;
    if (R2 > 0 && L.lazy) {
        // giant steps: key products of all k2 summed over Q*P, one ModDown; sigma(c0) terms summed
        u64 *U, *usum, *s0, *acc;
        ResMap dm{};
        dm.per = k;
        dm.ngrp = R2;
        dm.off = 3L * k;                // k2 = 1, c1
        dm.gstride = 2L * k;
        dm.ostride = (long)t2 * 2 * k;
        for (int i = 0; i < k; ++i) dm.prime[i] = i;
        CTL_TRY(keyswitch_raise(c, st, k, B, R2, inner, dm, false, ks, gal2.data(), gal2.data(), &U));
        CTL_TRY(slot(c, S_ROT2, (size_t)B * 2 * (k + 1) * N, st, &usum));
        CTL_TRY(slot(c, S_TENSOR, (size_t)B * ctw, st, &s0));
        CTL_TRY(slot(c, S_SUM, (size_t)B * ctw, st, &acc));
        GalList one{}, gl{};
        for (int r = 0; r < kMaxKeysPerLaunch; ++r) one.g[r] = 1;
        for (int r = 0; r < R2; ++r) gl.g[r] = gal2[r];
        const long ext = 2L * (k + 1) * N;
        { CTL_PROF(F_ADD, (double)B * ext, 0.0); launch_sum_gather(logn, usum, ext, nullptr, 0, U, (long)R2 * ext, ext, R2, k + 1, true, 3, one, B, c->hp.nq, c->tab, st); }
        { CTL_PROF(F_ADD, (double)B * ctw, 0.0); launch_sum_gather(logn, s0, ctw, inner, (long)t2 * ctw, inner + ctw, (long)t2 * ctw, ctw, R2, k, false, 1, gl, B, c->hp.nq, c->tab, st); }
        DropAdd add{};
        add.base = s0;
        add.sb = ctw;
        add.sc = (long)k * N;
        add.R = 1;
        add.mask = 3;
        add.gal[0] = 1;
        CTL_TRY(keyswitch_lower(c, st, k, B * 2, usum, add, acc));
        sum = acc;
    } else if (R2 > 0) {
        // giant steps rot_{k2 t1}(inner_k2), k2 = 1..t2-1, one key switch each, then the sum
        u64 *rot2, *acc;
        CTL_TRY(slot(c, S_ROT2, (size_t)B * R2 * ctw, st, &rot2));
        CTL_TRY(slot(c, S_SUM, (size_t)B * ctw, st, &acc));
        ResMap dm{};
        dm.per = k;
        dm.ngrp = R2;
        dm.off = 3L * k;                // k2 = 1, c1
        dm.gstride = 2L * k;
        dm.ostride = (long)t2 * 2 * k;
        for (int i = 0; i < k; ++i) dm.prime[i] = i;
        DropAdd add{};
        add.base = inner + ctw;         // inner_1, c0
        add.sb = (long)t2 * ctw;
        add.sr = ctw;
        add.R = R2;
        add.mask = 1;
        for (int r = 0; r < R2; ++r) add.gal[r] = gal2[r];
        CTL_TRY(keyswitch_batch(c, st, k, B, R2, inner, dm, false, ks, gal2.data(), gal2.data(), add, rot2));
        { CTL_PROF(F_ADD, 2.0 * B * k * N, 0.0); launch_add_terms(logn, inner, (long)t2 * ctw, rot2, (long)R2 * ctw, ctw, R2, acc, B, k, c->tab, st); }
        CTL_TRY(check_launch());
        sum = acc;
    }
    Site s(c, kKeepLayer, "rescale");
    return rescale_batch(c, st, k, B, sum, out);
}

// The model's layers in order on [B][2][n_q][N] -> [B][2][k_out][N], through three rotating
// context buffers (a layer's input may be the caller's `in`, its output never aliases it).
int forward_batch(ctl_ctx *c, hipStream_t st, const ctl_model *m, const KeySet &ks, int B, const u64 *in,
                  u64 *out) {
    const long N = c->hp.n;
    const size_t words = (size_t)B * 2 * c->hp.nq * N;
    u64 *bufs[3];
    CTL_TRY(slot(c, S_FWD_A, words, st, &bufs[0]));
    CTL_TRY(slot(c, S_FWD_B, words, st, &bufs[1]));
    CTL_TRY(slot(c, S_FWD_C, words, st, &bufs[2]));
    const u64 *cur = in;
    int ci = 2;                                   // the next result goes to bufs[(ci + 1) % 3]
    auto next = [&]() { ci = (ci + 1) % 3; return bufs[ci]; };
    const int L = (int)m->layers.size();
    for (int l = 0; l < L; ++l) {
        const LayerPlan &P = m->layers[l];
        Site layer(c, l, "");
        if (P.rep_before) {
            Site s(c, kKeepLayer, "replicate");
            u64 *dst = next();
            CTL_TRY(replicate_batch(c, st, ks, P.k, B, P.rep_before, cur, dst));
            cur = dst;
        }
        const bool last = l + 1 == L;
        u64 *dst = last ? out : next();
        CTL_TRY(dense_batch(c, st, m, l, ks, B, cur, dst));
        cur = dst;
        if (last) break;
        if (P.act == CTL_ACT_SQUARE) {
            Site s(c, kKeepLayer, "square");
            u64 *d2 = next();
            CTL_TRY(square_batch(c, st, ks, P.k - 1, B, cur, d2));
            cur = d2;
        } else if (P.act == CTL_ACT_POLY3) {
            Site s(c, kKeepLayer, "cubic");
            u64 *d2 = next();
            CTL_TRY(poly3_batch(c, st, ks, P.k - 1, B, P.act_scale_in, P.act_coef, cur, d2));
            cur = d2;
        }
    }
    return CTL_OK;
}

// ---------------------------------------------------------------- model planning
int plan_model(const ctl_ctx *c, const ctl_layer_desc *layers, int n_layers, const ctl_model_opts *opts,
               ctl_model *m) {
    if (!layers || n_layers < 1 || n_layers > 8) return fail(CTL_EINVAL, "1..8 layers supported");
    int tmax = 0;
    for (int l = 0; l < n_layers; ++l) {
        const ctl_layer_desc &d = layers[l];
        LayerPlan L;
        L.kind = d.kind;
        L.n_in = d.n_in;
        L.n_out = d.n_out;
        L.act = d.act;
        L.f = d.f;
        if (d.n_in < 1 || d.n_out < 1) return fail(CTL_EINVAL, "layer widths must be positive");
        if (l > 0 && d.n_in != layers[l - 1].n_out) return fail(CTL_EINVAL, "layer widths do not chain");
        if (l > 0 && layers[l - 1].kind == CTL_LAYER_AVGPOOL && d.kind != CTL_LAYER_DENSE)
            return fail(CTL_EINVAL, "an average pool must be followed by a dense layer");
        if (d.flags & ~(CTL_LAYER_LAZY_GIANT | CTL_LAYER_BABY_QP)) return fail(CTL_EINVAL, "unknown layer flag");
        if ((d.flags & CTL_LAYER_LAZY_GIANT) && d.kind != CTL_LAYER_DENSE)
            return fail(CTL_EINVAL, "CTL_LAYER_LAZY_GIANT applies to dense layers");
        L.qp = (d.flags & CTL_LAYER_BABY_QP) != 0;
        if (d.kind == CTL_LAYER_DENSE) {
            L.in_off = (l > 0 && layers[l - 1].kind == CTL_LAYER_AVGPOOL) ? layers[l - 1].f - 1 : 0;
            L.t = std::max(L.in_off + d.n_in, d.n_out);
            if (d.t1 < 1 || L.t % d.t1) return fail(CTL_EINVAL, "t1 must divide the padded width");
            L.t1 = d.t1;
            L.t2 = L.t / d.t1;
            L.lazy = L.qp || (d.flags & CTL_LAYER_LAZY_GIANT) != 0;
            for (int j = 1; j < L.t1; ++j) L.rots1.push_back(j);
        } else if (d.kind == CTL_LAYER_CONV1D) {
            if (d.f < 1 || d.f % 2 == 0 || d.f > 2 * d.n_in - 1)
                return fail(CTL_EINVAL, "convolution size must be odd and below twice the width");
            if (d.n_out != d.n_in) return fail(CTL_EINVAL, "a 'same' convolution keeps the width");
            L.t = d.n_in;
            L.t1 = d.f;
            L.t2 = 1;
            const int h = (d.f - 1) / 2;
            for (int r = -h; r <= h; ++r)
                if (r) L.rots1.push_back(r);
        } else if (d.kind == CTL_LAYER_AVGPOOL) {
            if (d.f < 1 || d.f > d.n_in) return fail(CTL_EINVAL, "pool size must lie in 1..n_in");
            if (d.n_out != d.n_in - d.f + 1) return fail(CTL_EINVAL, "a stride-1 pool gives n_in - f + 1 outputs");
            L.t = d.n_in;
            L.t1 = d.f;
            L.t2 = 1;
            for (int i = 1; i < d.f; ++i) L.rots1.push_back(-i);
        } else {
            return fail(CTL_EINVAL, "unknown layer kind");
        }
        L.nb = L.t1 * L.t2;
        if (d.act != CTL_ACT_NONE && d.act != CTL_ACT_SQUARE && d.act != CTL_ACT_POLY3)
            return fail(CTL_EINVAL, "unknown activation");
        if (d.act != CTL_ACT_NONE && l == n_layers - 1)
            return fail(CTL_EINVAL, "the activation is applied between layers only");
        for (int i = 0; i < 4; ++i) L.act_coef[i] = d.coef[i];
        tmax = std::max(tmax, L.t);
        m->layers.push_back(L);
    }
    m->block = 2 * tmax;
    if (opts && opts->block) {
        if (opts->block < 2 * tmax || opts->block > c->hp.n / 2)
            return fail(CTL_EINVAL, "block must lie in [2 t_max, N/2]");
        m->block = opts->block;
    }
    m->items = (c->hp.n / 2) / m->block;
    if (m->items < 1) return fail(CTL_EINVAL, "layers wider than N/4 slots");
    int k = c->hp.nq;
    if (opts && opts->k_in) {
        if (opts->k_in < 2 || opts->k_in > c->hp.nq) return fail(CTL_ELEVEL, "k_in out of range");
        k = opts->k_in;
    }
    double scale = std::ldexp(1.0, c->hp.log2_scale);
    if (opts && opts->scale_in != 0.0) {
        if (!(opts->scale_in > 0.0) || !std::isfinite(opts->scale_in)) return fail(CTL_ESCALE, "bad scale_in");
        scale = opts->scale_in;
    }
    m->scale_in = scale;
    std::vector<int32_t> rots;
    int doubled = m->layers[0].t;            // the client encodes [x | x] with the first layer's width
    for (int l = 0; l < n_layers; ++l) {
        LayerPlan &L = m->layers[l];
        if (L.kind != CTL_LAYER_AVGPOOL && doubled != L.t) {
            L.rep_before = L.t;
            rots.push_back(-L.t);
            doubled = L.t;
        }
        if (k < 2) return fail(CTL_ELEVEL, "modulus chain exhausted at layer " + std::to_string(l));
        L.k = k;
        L.pt_scale = (double)c->hp.mods[k - 1];
        // the 128-bit accumulation of t1 products must not overflow
        for (int i = 0; i < k; ++i) {
            const u128 sq = (u128)(c->hp.mods[i] - 1) * (c->hp.mods[i] - 1);
            if (sq > (~(u128)0) / (u128)L.t1) return fail(CTL_EPARAM, "t1 too large for the prime sizes");
        }
        for (long r : L.rots1) rots.push_back((int32_t)r);
        for (int k2 = 1; k2 < L.t2; ++k2) rots.push_back(k2 * L.t1);
        k -= 1;                                  // one rescale, scale unchanged
        doubled = L.kind == CTL_LAYER_CONV1D ? L.t : 0;
        L.act_scale_in = scale;
        if (L.act == CTL_ACT_SQUARE) {
            if (k < 2) return fail(CTL_ELEVEL, "modulus chain exhausted before x^2");
            scale = scale * scale / (double)c->hp.mods[k - 1];
            k -= 1;
        } else if (L.act == CTL_ACT_POLY3) {
            if (k < 3) return fail(CTL_ELEVEL, "modulus chain exhausted before the cubic activation");
            if (!poly3_consts_ok(c, k, scale, L.act_coef)) return fail(CTL_ESCALE, "activation constant out of range");
            int64_t C[4];
            scale = poly3_consts(c, k, scale, L.act_coef, C);
            k -= 2;
        }
    }
    if (k < 1) return fail(CTL_ELEVEL, "modulus chain exhausted");
    m->k_out = k;
    m->scale_out = scale;
    std::set<int32_t> seen;
    for (int32_t r : rots)
        if (seen.insert(r).second) m->rotations.push_back(r);
    return CTL_OK;
}

// diag'_i of Eq. (1) on its support: in every item block, slot k2 t1 + s holds M[s][(s + i) mod t],
// M the t x t matrix with W in rows 0..n_out-1 and columns in_off..in_off+n_in-1.
void diag_slots(const ctl_model *m, const LayerPlan &L, const double *W, int i, int half_n, double *z) {
    std::fill(z, z + half_n, 0.0);
    const int k2 = i / L.t1;
    for (int b = 0; b < m->items; ++b) {
        double *blk = z + (long)b * m->block + (long)k2 * L.t1;
        for (int s = 0; s < L.t; ++s) {
            const int col = (s + i) % L.t - L.in_off;
            blk[s] = (s < L.n_out && col >= 0 && col < L.n_in) ? W[(long)s * L.n_in + col] : 0.0;
        }
    }
}

// Bank entry j of a convolution multiplies rot_r(x), r = 0 for j = 0 and rots1[j-1] otherwise; it
// carries tap r + (f-1)/2 on both halves of every block, where x[s + r] lies inside the width.
int conv_tap(const LayerPlan &L, int j) { return (j == 0 ? 0 : (int)L.rots1[j - 1]) + (L.f - 1) / 2; }

void conv_slots(const ctl_model *m, const LayerPlan &L, const double *taps, int j, int half_n, double *z) {
    std::fill(z, z + half_n, 0.0);
    const int i = conv_tap(L, j), r = i - (L.f - 1) / 2, w = L.n_in;
    for (int b = 0; b < m->items; ++b)
        for (int h = 0; h < 2; ++h) {
            double *blk = z + (long)b * m->block + (long)h * w;
            for (int s = 0; s < w; ++s) blk[s] = (s + r >= 0 && s + r < w) ? taps[i] : 0.0;
        }
}

// The pooling plaintext: 1/f on the valid outputs (slots f-1 .. n_in-1 of each block), 0 elsewhere.
void pool_slots(const ctl_model *m, const LayerPlan &L, int half_n, double *z) {
    std::fill(z, z + half_n, 0.0);
    for (int b = 0; b < m->items; ++b)
        for (int s = L.f - 1; s < L.n_in; ++s) z[(long)b * m->block + s] = 1.0 / L.f;
}

// Plaintexts a caller of the raw loader passes for a layer: dense t, convolution f, pool 1.
int raw_count(const LayerPlan &L) {
    return L.kind == CTL_LAYER_DENSE ? L.t : L.kind == CTL_LAYER_CONV1D ? L.f : 1;
}

int encode_to_int(const ctl_ctx *c, const double *z, double scale, int64_t *out) {
    const int n = c->hp.n;
    std::vector<double> m(n);
    c->enc->encode_real(z, m.data());
    for (int i = 0; i < n; ++i) {
        const double v = std::nearbyint(scale * m[i]);
        if (!(std::fabs(v) < 4611686018427387904.0)) return fail(CTL_ESCALE, "encoded coefficient reaches 2^62");
        out[i] = (int64_t)v;
    }
    return CTL_OK;
}

// Upload signed coefficients [G][N] and transform them to primes 0..k-1: out [G][k][N].
// G signed polynomials -> [G][k][N] NTT form over q_0..q_{k-1} (ext: [G][k+1][N], last row mod P).
int upload_ints(ctl_ctx *c, hipStream_t st, const int64_t *host, int G, int k, u64 *out, bool ext = false) {
    const long N = c->hp.n;
    u64 *stage;
    CTL_TRY(slot(c, S_MISC, (size_t)G * N, st, &stage));
    CTL_HIP(hipMemcpyAsync(stage, host, (size_t)G * N * 8, hipMemcpyHostToDevice, st));
    PrimeList pl{};
    pl.n = k;
    for (int i = 0; i < k; ++i) pl.idx[i] = i;
    if (ext) pl.idx[pl.n++] = c->hp.nq;
    launch_int_ntt(c->hp.logn, reinterpret_cast<const int64_t *>(stage), out, G, pl, c->tab, st);
    CTL_TRY(check_launch());
    CTL_HIP(hipStreamSynchronize(st));
    return CTL_OK;
}

int bank_rows(const LayerPlan &L) { return L.k + (L.qp ? 1 : 0); }

int load_banks(ctl_ctx *c, ctl_model *m, const std::vector<std::vector<int64_t>> *ints,
               const double *const *weights) {
    hipStream_t st = nullptr;
    const int n = c->hp.n;
    for (size_t l = 0; l < m->layers.size(); ++l) {
        const LayerPlan &L = m->layers[l];
        const int rows = bank_rows(L);
        u64 *bank = static_cast<u64 *>(dev_alloc(c, (size_t)L.nb * rows * n * 8, st));
        if (!bank) return fail(CTL_ENOMEM, "plaintext bank allocation failed");
        m->banks.push_back(bank);
        const int chunk = 32;
        std::vector<int64_t> buf((size_t)chunk * n);
        std::vector<double> z(n / 2);
        for (int i0 = 0; i0 < L.nb; i0 += chunk) {
            const int cnt = std::min(chunk, L.nb - i0);
            for (int i = 0; i < cnt; ++i) {
                const int j = i0 + i;
                // the caller's plaintext for bank entry j (dense: j; convolution: its tap; pool: the one)
                const int src = L.kind == CTL_LAYER_DENSE ? j : L.kind == CTL_LAYER_CONV1D ? conv_tap(L, j) : 0;
                if (ints) {
                    std::memcpy(&buf[(size_t)i * n], (*ints)[l].data() + (size_t)src * n, (size_t)n * 8);
                } else {
                    if (L.kind == CTL_LAYER_DENSE) diag_slots(m, L, weights[l], j, n / 2, z.data());
                    else if (L.kind == CTL_LAYER_CONV1D) conv_slots(m, L, weights[l], j, n / 2, z.data());
                    else pool_slots(m, L, n / 2, z.data());
                    CTL_TRY(encode_to_int(c, z.data(), L.pt_scale, &buf[(size_t)i * n]));
                }
            }
            CTL_TRY(upload_ints(c, st, buf.data(), cnt, L.k, bank + (size_t)i0 * rows * n, L.qp));
        }
    }
    return CTL_OK;
}

int make_model(ctl_ctx *c, const ctl_layer_desc *layers, int n_layers, const int64_t *const *pts,
               const double *const *weights, const ctl_model_opts *opts, ctl_model **out) {
    if (!c || !out) return fail(CTL_EINVAL, "null argument");
    std::unique_ptr<ctl_model> m(new (std::nothrow) ctl_model());
    if (!m) return fail(CTL_ENOMEM, "host allocation failed");
    m->ctx = c;
    CTL_TRY(plan_model(c, layers, n_layers, opts, m.get()));
    CTL_HIP(hipSetDevice(c->device));
    int rc;
    if (pts) {
        std::vector<std::vector<int64_t>> ints(n_layers);
        for (int l = 0; l < n_layers; ++l) {
            if (!pts[l]) return fail(CTL_EINVAL, "null plaintext array");
            const size_t cnt = (size_t)raw_count(m->layers[l]) * c->hp.n;
            for (size_t x = 0; x < cnt; ++x)
                if (pts[l][x] >= (int64_t)(1ull << 62) || pts[l][x] <= -(int64_t)(1ull << 62))
                    return fail(CTL_ESCALE, "plaintext coefficient out of range");
            ints[l].assign(pts[l], pts[l] + cnt);
        }
        rc = load_banks(c, m.get(), &ints, nullptr);
    } else {
        for (int l = 0; l < n_layers; ++l)
            if (!weights[l] && m->layers[l].kind != CTL_LAYER_AVGPOOL) return fail(CTL_EINVAL, "null weights");
        rc = load_banks(c, m.get(), nullptr, weights);
    }
    if (rc != CTL_OK) {
        for (u64 *b : m->banks) dev_free(c, b, nullptr);
        return rc;
    }
    ctx_retain(c);
    *out = m.release();
    return CTL_OK;
}

// c1 = a of a seeded symmetric ciphertext: uniform NTT values over q_0..q_{nq-1}, prime by prime.
void seeded_a(const ctl_ctx *ctx, uint64_t seed, std::vector<u64> &a) {
    const int n = ctx->hp.n, nq = ctx->hp.nq;
    a.resize((size_t)nq * n);
    Stream sa(seed, TAG_SYM_A, 0);
    for (int i = 0; i < nq; ++i)
        for (int x = 0; x < n; ++x) a[(size_t)i * n + x] = sa.uniform(ctx->hp.mods[i]);
}

// ---------------------------------------------------------------- wire format
constexpr uint8_t kMagic[4] = {'C', 'T', 'L', '1'};
constexpr int kHeader = 24;

u64 params_digest(const HostParams &h) {             // FNV-1a over the primes, little-endian words
    u64 d = 1469598103934665603ull;
    for (int i = 0; i < h.np; ++i)
        for (int b = 0; b < 8; ++b) {
            d ^= (h.mods[i] >> (8 * b)) & 0xff;
            d *= 1099511628211ull;
        }
    return d;
}

int bits_of(u64 q) { int b = 0; while (b < 64 && (q >> b)) ++b; return b; }

u64 packed_bytes(const HostParams &h, int k, int n_poly) {
    u64 bits = 0;
    for (int i = 0; i < k; ++i) bits += (u64)bits_of(h.mods[i]) * h.n;
    return kHeader + (u64)n_poly * bits / 8;
}

void put_u64(uint8_t *p, u64 v) { for (int b = 0; b < 8; ++b) p[b] = (uint8_t)(v >> (8 * b)); }
u64 get_u64(const uint8_t *p) { u64 v = 0; for (int b = 0; b < 8; ++b) v |= (u64)p[b] << (8 * b); return v; }

}  // namespace

// =============================================================================== exported API
extern "C" {

const char *ctl_last_error(void) { return g_err.c_str(); }

int ctl_params_primes(const ctl_params *params, uint64_t *primes_out, int *n_out) {
    if (!params || !primes_out || !n_out) return fail(CTL_EINVAL, "null argument");
    HostParams h;
    CTL_TRY(derive_params(params, &h, &g_err));
    for (int i = 0; i < h.np; ++i) primes_out[i] = h.mods[i];
    *n_out = h.np;
    return CTL_OK;
}

int ctl_galois_elt(const ctl_params *params, int rotation, uint64_t *g_out) {
    if (!params || !g_out) return fail(CTL_EINVAL, "null argument");
    if (params->log2n < 12 || params->log2n > 14) return fail(CTL_EPARAM, "log2n must be 12, 13 or 14");
    *g_out = galois_elt(params->log2n, rotation);
    return CTL_OK;
}

int ctl_sample(const ctl_params *params, uint64_t seed, uint32_t tag, uint64_t index, int kind,
               uint64_t modulus, int n, int64_t *out) {
    if (!params || !out || n < 0) return fail(CTL_EINVAL, "bad argument");
    HostParams h;
    CTL_TRY(derive_params(params, &h, &g_err));
    Stream s(seed, tag, index);
    if (kind == 0) s.ternary(n, out);
    else if (kind == 1) s.gaussian(h.cdt, n, out);
    else if (kind == 2) {
        if (modulus < 2) return fail(CTL_EINVAL, "modulus must be at least 2");
        for (int i = 0; i < n; ++i) out[i] = (int64_t)s.uniform(modulus);
    } else return fail(CTL_EINVAL, "unknown sampler kind");
    return CTL_OK;
}

int ctl_ctx_create(const ctl_params *params, int device, ctl_ctx **ctx_out) {
    if (!params || !ctx_out) return fail(CTL_EINVAL, "null argument");
    std::unique_ptr<ctl_ctx> c(new (std::nothrow) ctl_ctx());
    if (!c) return fail(CTL_ENOMEM, "host allocation failed");
    CTL_TRY(derive_params(params, &c->hp, &g_err));
    c->device = device;
    CTL_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    CTL_HIP(hipGetDeviceProperties(&prop, device));
    c->tab.cus = prop.multiProcessorCount;
    c->tab.lds_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    const size_t lds_need = (size_t)(c->hp.n + c->hp.n / 32) * 8;
    if (prop.sharedMemPerBlock < lds_need && prop.maxSharedMemoryPerMultiProcessor < lds_need)
        return fail(CTL_EPARAM, "device LDS too small for N = " + std::to_string(c->hp.n));
    const int n = c->hp.n, np = c->hp.np;
    // tables: tw, tws, itw, itws [np][N]; PrimeConst [np]; CrossConst [kMaxMods][kMaxMods]
    const size_t tw_words = (size_t)np * n;
    const size_t bytes = 4 * tw_words * 8 + sizeof(PrimeConst) * kMaxMods + sizeof(CrossConst) * kMaxMods * kMaxMods;
    std::vector<unsigned char> host(bytes, 0);
    u64 *tw = reinterpret_cast<u64 *>(host.data());
    u64 *tws = tw + tw_words, *itw = tws + tw_words, *itws = itw + tw_words;
    PrimeConst *pc = reinterpret_cast<PrimeConst *>(itws + tw_words);
    CrossConst *cross = reinterpret_cast<CrossConst *>(pc + kMaxMods);
    std::vector<u64> pw(n), ipw(n);
    for (int i = 0; i < np; ++i) {
        const u64 q = c->hp.mods[i], psi = c->hp.psi[i], ipsi = h_invmod(psi, q);
        pw[0] = ipw[0] = 1;
        for (int e = 1; e < n; ++e) {
            pw[e] = h_mulmod(pw[e - 1], psi, q);
            ipw[e] = h_mulmod(ipw[e - 1], ipsi, q);
        }
        const bool fp = q < kFpPrimeLimit;
        c->tab.host_fp[i] = fp ? 1 : 0;
        c->tab.host_lt60[i] = c->hp.mods[i] < (1ull << 60) ? 1 : 0;
        for (int m = 0; m < n; ++m) {
            unsigned r = 0;
            for (int b = 0; b < c->hp.logn; ++b) r |= ((m >> b) & 1u) << (c->hp.logn - 1 - b);
            tw[(size_t)i * n + m] = pw[r];
            itw[(size_t)i * n + m] = ipw[r];
            if (fp) {
                // FP64 path: the companion slots carry the twiddles as doubles (exact below 2^53)
                const double a = (double)pw[r], b = (double)ipw[r];
                std::memcpy(&tws[(size_t)i * n + m], &a, 8);
                std::memcpy(&itws[(size_t)i * n + m], &b, 8);
            } else {
                tws[(size_t)i * n + m] = h_shoup(pw[r], q);
                itws[(size_t)i * n + m] = h_shoup(ipw[r], q);
            }
        }
        PrimeConst &p = pc[i];
        p.q = q;
        p.q2 = 2 * q;
        p.r64 = (u64)(((u128)1 << 64) % q);
        p.r64s = h_shoup(p.r64, q);
        p.ones = (u64)(((u128)1 << 64) / q);
        p.ninv = h_invmod((u64)n % q, q);
        p.ninvs = h_shoup(p.ninv, q);
        p.qn = 0 - q;
        p.nq2 = 0 - 2 * q;
        p.r60 = q < (1ull << 60) ? (1ull << 60) % q : 1ull << 60;
        p.r60s = q < (1ull << 60) ? h_shoup(p.r60, q) : 0;
        p.fp = fp ? 1 : 0;
        p.pad_ = 0;
        p.qd = (double)q;
        p.qinv = 1.0 / (double)q;
        p.ninvd = (double)p.ninv;
        c->pc.push_back(p);
    }
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            CrossConst &cc = cross[i * kMaxMods + j];
            const u64 qi = c->hp.mods[i], qj = c->hp.mods[j];
            cc.qj_mod_qi = qj % qi;
            cc.inv = i == j ? 0 : h_invmod(qj % qi, qi);
            cc.invs = h_shoup(cc.inv, qi);
            cc.invd = (double)cc.inv;
        }
    void *dmem = nullptr;
    CTL_HIP(hipMalloc(&dmem, bytes));
    if (hipMemcpy(dmem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dmem);
        return fail(CTL_EHIP, "table upload failed");
    }
    c->tables_mem = dmem;
    u64 *d = static_cast<u64 *>(dmem);
    c->tab.tw = d;
    c->tab.tws = d + tw_words;
    c->tab.itw = d + 2 * tw_words;
    c->tab.itws = d + 3 * tw_words;
    c->tab.pc = reinterpret_cast<const PrimeConst *>(d + 4 * tw_words);
    c->tab.cross = reinterpret_cast<const CrossConst *>(c->tab.pc + kMaxMods);
    if (kernels_prepare(c->hp.logn) != hipSuccess) {
        (void)hipFree(dmem);
        return fail(CTL_EHIP, "setting the LDS limit of the NTT kernels failed");
    }
    if (scratch_device_address(device, &c->scratch) != hipSuccess) {
        (void)hipFree(dmem);
        return fail(CTL_EHIP, "looking up the scratch array's device address failed");
    }
    c->enc.reset(new Encoder(c->hp.logn));
    *ctx_out = c.release();
    return CTL_OK;
}

int ctl_ctx_free(ctl_ctx *ctx) {
    if (!ctx) return CTL_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (int s = 0; s < S_COUNT; ++s) dev_free(ctx, ctx->slot_ptr[s], nullptr);
    for (int s = 0; s < S_COUNT; ++s) {
        ctx->slot_ptr[s] = nullptr;
        ctx->slot_bytes[s] = 0;
    }
    for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
    ctx->prof_ev.clear();
    ctx->prof_fam.clear();
    ctx->prof_work.clear();
    ctx->prof_fp.clear();
    ctx->prof_bytes.clear();
    ctx->prof_layer_v.clear();
    ctx->prof_phase_v.clear();
    ctx->prof_used = 0;
    ctx_release(ctx);              // the tables stay until the last handle made here is freed
    return CTL_OK;
}

int ctl_ctx_primes(const ctl_ctx *ctx, uint64_t *primes_out, int *n_out) {
    if (!ctx || !primes_out || !n_out) return fail(CTL_EINVAL, "null argument");
    for (int i = 0; i < ctx->hp.np; ++i) primes_out[i] = ctx->hp.mods[i];
    *n_out = ctx->hp.np;
    return CTL_OK;
}

int ctl_set_allocator(ctl_ctx *ctx, ctl_alloc_fn alloc, ctl_free_fn free_fn, void *user) {
    if (!ctx) return fail(CTL_EINVAL, "null context");
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(CTL_EINVAL, "give both alloc and free");
    for (int s = 0; s < S_COUNT; ++s)
        if (ctx->slot_ptr[s]) return fail(CTL_EINVAL, "allocator must be set before the first allocation");
    ctx->alloc = alloc;
    ctx->free_fn = free_fn;
    ctx->user = user;
    return CTL_OK;
}

int ctl_workspace_freeze(ctl_ctx *ctx, int frozen) {
    if (!ctx) return fail(CTL_EINVAL, "null context");
    ctx->ws_frozen = frozen != 0;
    return CTL_OK;
}

int ctl_knob_set(ctl_ctx *ctx, int knob, int value) {
    if (!ctx) return fail(CTL_EINVAL, "null context");
    switch (knob) {
        case CTL_KNOB_MAC_CHUNK:
            if (value < 1 || value > 16) return fail(CTL_EINVAL, "MAC chunk cap must lie in 1..16");
            ctx->knobs.mac_chunk_cap = value;
            return CTL_OK;
        case CTL_KNOB_MAC_CTS:
            if (value < 1 || value > 16) return fail(CTL_EINVAL, "ciphertexts per MAC workgroup must lie in 1..16");
            ctx->knobs.mac_cts = value;
            return CTL_OK;
        case CTL_KNOB_KEYIP_XCD:
            if (value != 0 && value != 1) return fail(CTL_EINVAL, "key-product numbering is 0 or 1");
            ctx->knobs.keyip_xcd = value;
            return CTL_OK;
        case CTL_KNOB_MAC_DIRECT:
            if (value < 0 || value > 64) return fail(CTL_EINVAL, "direct-MAC batch limit must lie in 0..64");
            ctx->knobs.mac_direct_max = value;
            return CTL_OK;
        case CTL_KNOB_NTT_XCD:
            if (value != 0 && value != 1) return fail(CTL_EINVAL, "ModUp/ModDown numbering is 0 or 1");
            ctx->knobs.ntt_xcd = value;
            return CTL_OK;
        case CTL_KNOB_MAC_LIMB:
            if (value != 0 && value != 1) return fail(CTL_EINVAL, "the limb MAC switch is 0 or 1");
            ctx->knobs.mac_limb = value;
            return CTL_OK;
        case CTL_KNOB_KEYIP_RR:
            if (value < 1 || value > 8) return fail(CTL_EINVAL, "rotations per key-product workgroup must lie in 1..8");
            ctx->knobs.keyip_rr = value;
            return CTL_OK;
        case CTL_KNOB_NTT_SPLIT:
            if (value < 0 || value > 4096) return fail(CTL_EINVAL, "the split threshold must lie in 0..4096");
            ctx->knobs.ntt_split = value;
            return CTL_OK;
        case CTL_KNOB_NTT_LOOP:
            if (value < 0 || value > 64) return fail(CTL_EINVAL, "the loop threshold must lie in 0..64");
            ctx->knobs.ntt_loop = value;
            return CTL_OK;
        case CTL_KNOB_FUSE_RESCALE:
            if (value != 0 && value != 1) return fail(CTL_EINVAL, "the ModDown + rescale switch is 0 or 1");
            ctx->knobs.fuse_rescale = value;
            return CTL_OK;
        default:
            return fail(CTL_EINVAL, "unknown knob");
    }
}

int ctl_knob_get(const ctl_ctx *ctx, int knob, int *value) {
    if (!ctx || !value) return fail(CTL_EINVAL, "null argument");
    switch (knob) {
        case CTL_KNOB_MAC_CHUNK: *value = ctx->knobs.mac_chunk_cap; return CTL_OK;
        case CTL_KNOB_MAC_CTS: *value = ctx->knobs.mac_cts; return CTL_OK;
        case CTL_KNOB_KEYIP_XCD: *value = ctx->knobs.keyip_xcd; return CTL_OK;
        case CTL_KNOB_MAC_DIRECT: *value = ctx->knobs.mac_direct_max; return CTL_OK;
        case CTL_KNOB_NTT_XCD: *value = ctx->knobs.ntt_xcd; return CTL_OK;
        case CTL_KNOB_MAC_LIMB: *value = ctx->knobs.mac_limb; return CTL_OK;
        case CTL_KNOB_KEYIP_RR: *value = ctx->knobs.keyip_rr; return CTL_OK;
        case CTL_KNOB_NTT_SPLIT: *value = ctx->knobs.ntt_split; return CTL_OK;
        case CTL_KNOB_NTT_LOOP: *value = ctx->knobs.ntt_loop; return CTL_OK;
        case CTL_KNOB_FUSE_RESCALE: *value = ctx->knobs.fuse_rescale; return CTL_OK;
        default: return fail(CTL_EINVAL, "unknown knob");
    }
}

int ctl_workspace_bytes(const ctl_ctx *ctx, uint64_t *bytes_out) {
    if (!ctx || !bytes_out) return fail(CTL_EINVAL, "null argument");
    uint64_t t = 0;
    for (int s = 0; s < S_COUNT; ++s) t += ctx->slot_bytes[s];
    *bytes_out = t;
    return CTL_OK;
}

int ctl_profile_enable(ctl_ctx *ctx, int enable) {
    if (!ctx) return fail(CTL_EINVAL, "null context");
    ctx->prof_on = enable != 0;
    if (ctx->prof_on) ctx->prof_used = 0;
    return CTL_OK;
}

int ctl_profile_families(void) { return F_COUNT; }

const char *ctl_profile_family_name(int family) {
    return family >= 0 && family < F_COUNT ? kFamilyNames[family] : "";
}

int ctl_profile_read(ctl_ctx *ctx, int family, int *launches_out, double *total_ms_out, double *work_out,
                     double *fp_work_out) {
    if (!ctx || !launches_out || !total_ms_out || !work_out || !fp_work_out) return fail(CTL_EINVAL, "null argument");
    if (family < 0 || family >= F_COUNT) return fail(CTL_EINVAL, "unknown kernel family");
    int cnt = 0;
    double tot = 0.0, work = 0.0, fpw = 0.0;
    for (size_t i = 0; i < ctx->prof_used; ++i) {
        if (ctx->prof_fam[i] != family) continue;
        CTL_HIP(hipEventSynchronize(ctx->prof_ev[2 * i + 1]));
        float ms = 0.f;
        CTL_HIP(hipEventElapsedTime(&ms, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
        tot += ms;
        work += ctx->prof_work[i];
        fpw += ctx->prof_fp[i];
        ++cnt;
    }
    *launches_out = cnt;
    *total_ms_out = tot;
    *work_out = work;
    *fp_work_out = fpw;
    return CTL_OK;
}

int ctl_profile_read_bytes(ctl_ctx *ctx, int family, double *bytes_out) {
    if (!ctx || !bytes_out) return fail(CTL_EINVAL, "null argument");
    if (family < 0 || family >= F_COUNT) return fail(CTL_EINVAL, "unknown kernel family");
    double b = 0.0;
    for (size_t i = 0; i < ctx->prof_used; ++i)
        if (ctx->prof_fam[i] == family) b += ctx->prof_bytes[i];
    *bytes_out = b;
    return CTL_OK;
}

int ctl_profile_launches(ctl_ctx *ctx, int *n_out) {
    if (!ctx || !n_out) return fail(CTL_EINVAL, "null argument");
    *n_out = (int)ctx->prof_used;
    return CTL_OK;
}

int ctl_profile_launch(ctl_ctx *ctx, int i, int *family_out, double *ms_out, double *work_out, double *fp_work_out,
                       double *bytes_out, int *layer_out, const char **phase_out) {
    if (!ctx || !family_out || !ms_out || !work_out || !fp_work_out || !bytes_out || !layer_out || !phase_out)
        return fail(CTL_EINVAL, "null argument");
    if (i < 0 || (size_t)i >= ctx->prof_used) return fail(CTL_EINVAL, "launch record out of range");
    CTL_HIP(hipEventSynchronize(ctx->prof_ev[2 * i + 1]));
    float ms = 0.f;
    CTL_HIP(hipEventElapsedTime(&ms, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
    *family_out = ctx->prof_fam[i];
    *ms_out = ms;
    *work_out = ctx->prof_work[i];
    *fp_work_out = ctx->prof_fp[i];
    *bytes_out = ctx->prof_bytes[i];
    *layer_out = ctx->prof_layer_v[i];
    *phase_out = ctx->prof_phase_v[i];
    return CTL_OK;
}

int ctl_probe_valu(ctl_ctx *ctx, int kind, int iters, double *lane_ops_out, void *stream) {
    if (!ctx || !lane_ops_out || kind < 0 || kind > 3 || iters < 1 || iters > (1 << 24))
        return fail(CTL_EINVAL, "bad argument");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    hipDeviceProp_t prop;
    CTL_HIP(hipGetDeviceProperties(&prop, ctx->device));
    const int blocks = prop.multiProcessorCount * 8;       // 8 workgroups (32 waves) per CU
    u64 *out;
    CTL_TRY(slot(ctx, S_MISC, (size_t)blocks * 256, st, &out));
    hipEvent_t e0, e1;
    CTL_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CTL_EHIP, "event creation failed");
    }
    launch_probe(kind, std::max(1, iters / 16), 1, out, blocks, st);      // warm-up
    (void)hipEventRecord(e0, st);
    launch_probe(kind, iters, 2, out, blocks, st);
    (void)hipEventRecord(e1, st);
    const hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    const hipError_t e2 = e == hipSuccess ? hipEventElapsedTime(&ms, e0, e1) : e;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e2 != hipSuccess) return fail(CTL_EHIP, std::string("probe: ") + hipGetErrorString(e2));
    CTL_TRY(check_launch());
    *lane_ops_out = (double)blocks * 256 * iters * kProbeOpsPerThreadIter / (ms * 1e-3);
    return CTL_OK;
}

int ctl_ntt(ctl_ctx *ctx, uint64_t *dev, int n_res, const int32_t *prime_idx, int inverse, void *stream) {
    if (!ctx || (!dev && n_res) || (!prime_idx && n_res) || n_res < 0) return fail(CTL_EINVAL, "bad argument");
    for (int r = 0; r < n_res; ++r)
        if (prime_idx[r] < 0 || prime_idx[r] >= ctx->hp.np) return fail(CTL_EINVAL, "prime index out of range");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    const long N = ctx->hp.n;
    // a prime pattern that repeats with a short period runs as one launch
    int period = 0;
    for (int p = 1; p <= kMaxMods && p <= n_res && !period; ++p) {
        bool ok = true;
        for (int r = p; r < n_res && ok; ++r) ok = prime_idx[r] == prime_idx[r % p];
        if (ok) period = p;
    }
    if (period) {
        ResMap m = dense_map(period);
        for (int i = 0; i < period; ++i) m.prime[i] = prime_idx[i];
        u64 *p = reinterpret_cast<u64 *>(dev);
        Prof prof(ctx, inverse ? F_NTT_INV : F_NTT_FWD, st, n_res, fp_share(ctx, prime_idx, period));
        launch_ntt(ctx->hp.logn, inverse != 0, p, m, p, m, n_res, ctx->tab, ctx->knobs, st);
        return check_launch();
    }
    for (int r0 = 0; r0 < n_res; r0 += kMaxMods) {
        const int cnt = std::min(kMaxMods, n_res - r0);
        ResMap m{};
        m.per = cnt;
        m.ngrp = 1;
        m.off = 0;
        m.gstride = cnt;
        m.ostride = cnt;
        for (int i = 0; i < cnt; ++i) m.prime[i] = prime_idx[r0 + i];
        u64 *p = reinterpret_cast<u64 *>(dev) + (size_t)r0 * N;
        Prof prof(ctx, inverse ? F_NTT_INV : F_NTT_FWD, st, cnt, fp_share(ctx, prime_idx + r0, cnt));
        launch_ntt(ctx->hp.logn, inverse != 0, p, m, p, m, cnt, ctx->tab, ctx->knobs, st);
        CTL_TRY(check_launch());
    }
    return CTL_OK;
}

// ---------------------------------------------------------------- parity hooks
int ctl_ct_export(ctl_ctx *ctx, const uint64_t *ct, int k, int n_poly, int form, uint64_t *host_out, void *stream) {
    if (!ctx || !ct || !host_out || n_poly < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    if (form != CTL_FORM_NTT && form != CTL_FORM_COEFF) return fail(CTL_EINVAL, "unknown form");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    const size_t words = (size_t)n_poly * k * ctx->hp.n;
    const u64 *src = reinterpret_cast<const u64 *>(ct);
    if (form == CTL_FORM_COEFF) {
        u64 *tmp;
        CTL_TRY(slot(ctx, S_COEF2, words, st, &tmp));
        launch_ntt(ctx->hp.logn, true, src, dense_map(k), tmp, dense_map(k), n_poly * k, ctx->tab, ctx->knobs, st);
        CTL_TRY(check_launch());
        src = tmp;
    }
    CTL_HIP(hipMemcpyAsync(host_out, src, words * 8, hipMemcpyDeviceToHost, st));
    CTL_HIP(hipStreamSynchronize(st));
    return CTL_OK;
}

int ctl_ct_import(ctl_ctx *ctx, const uint64_t *host, int k, int n_poly, int form, uint64_t *ct_out, void *stream) {
    if (!ctx || !host || !ct_out || n_poly < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    if (form != CTL_FORM_NTT && form != CTL_FORM_COEFF) return fail(CTL_EINVAL, "unknown form");
    const long n = ctx->hp.n;
    for (int p = 0; p < n_poly; ++p)
        for (int i = 0; i < k; ++i)
            for (long x = 0; x < n; ++x)
                if (host[((size_t)p * k + i) * n + x] >= ctx->hp.mods[i])
                    return fail(CTL_EINVAL, "residue word not reduced modulo its prime");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    const size_t words = (size_t)n_poly * k * n;
    u64 *dst = reinterpret_cast<u64 *>(ct_out);
    if (form == CTL_FORM_COEFF) {
        u64 *tmp;
        CTL_TRY(slot(ctx, S_COEF2, words, st, &tmp));
        CTL_HIP(hipMemcpyAsync(tmp, host, words * 8, hipMemcpyHostToDevice, st));
        launch_ntt(ctx->hp.logn, false, tmp, dense_map(k), dst, dense_map(k), n_poly * k, ctx->tab, ctx->knobs, st);
        CTL_TRY(check_launch());
    } else {
        CTL_HIP(hipMemcpyAsync(dst, host, words * 8, hipMemcpyHostToDevice, st));
    }
    CTL_HIP(hipStreamSynchronize(st));
    return CTL_OK;
}

int ctl_pt_import(ctl_ctx *ctx, const int64_t *coeffs, int n_pt, int k, int ext, uint64_t *pt_out, void *stream) {
    if (!ctx || !coeffs || !pt_out || n_pt < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    const size_t cnt = (size_t)n_pt * ctx->hp.n;
    for (size_t x = 0; x < cnt; ++x)
        if (coeffs[x] >= (int64_t)(1ull << 62) || coeffs[x] <= -(int64_t)(1ull << 62))
            return fail(CTL_ESCALE, "plaintext coefficient out of range");
    CTL_HIP(hipSetDevice(ctx->device));
    return upload_ints(ctx, as_stream(stream), coeffs, n_pt, k, reinterpret_cast<u64 *>(pt_out), ext != 0);
}

// ---------------------------------------------------------------- keys
int ctl_keygen(ctl_ctx *ctx, uint64_t seed, const int32_t *rotations, int n_rot, int relin,
               ctl_sk **sk_out, ctl_pk **pk_out, ctl_evk **evk_out) {
    if (!ctx || (n_rot > 0 && !rotations) || n_rot < 0) return fail(CTL_EINVAL, "bad argument");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = nullptr;
    const int n = ctx->hp.n, nq = ctx->hp.nq, np = ctx->hp.np, logn = ctx->hp.logn;
    std::unique_ptr<ctl_sk> sk(new ctl_sk());
    sk->ctx = ctx;
    sk->s.resize(n);
    Stream(seed, TAG_SK, 0).ternary(n, sk->s.data());
    sk->d_s = static_cast<u64 *>(dev_alloc(ctx, (size_t)np * n * 8, st));
    if (!sk->d_s) return fail(CTL_ENOMEM, "secret key allocation failed");
    {
        u64 *stage;
        CTL_TRY(slot(ctx, S_MISC, (size_t)n, st, &stage));
        CTL_HIP(hipMemcpy(stage, sk->s.data(), (size_t)n * 8, hipMemcpyHostToDevice));
        PrimeList pl{};
        pl.n = np;
        for (int i = 0; i < np; ++i) pl.idx[i] = i;
        launch_int_ntt(logn, reinterpret_cast<const int64_t *>(stage), sk->d_s, 1, pl, ctx->tab, st);
        CTL_TRY(check_launch());
        CTL_HIP(hipStreamSynchronize(st));
    }
    std::unique_ptr<ctl_pk> pk;
    if (pk_out) {
        pk.reset(new ctl_pk());
        pk->ctx = ctx;
        pk->d_pk = static_cast<u64 *>(dev_alloc(ctx, (size_t)2 * nq * n * 8, st));
        if (!pk->d_pk) return fail(CTL_ENOMEM, "public key allocation failed");
        std::vector<u64> a((size_t)nq * n);
        Stream sa(seed, TAG_PK_A, 0);
        for (int i = 0; i < nq; ++i)
            for (int x = 0; x < n; ++x) a[(size_t)i * n + x] = sa.uniform(ctx->hp.mods[i]);
        std::vector<int64_t> e(n);
        Stream(seed, TAG_PK_E, 0).gaussian(ctx->hp.cdt, n, e.data());
        CTL_HIP(hipMemcpy(pk->d_pk + (size_t)nq * n, a.data(), (size_t)nq * n * 8, hipMemcpyHostToDevice));
        u64 *en;
        CTL_TRY(slot(ctx, S_COEF, (size_t)nq * n, st, &en));
        CTL_TRY(upload_ints(ctx, st, e.data(), 1, nq, en));
        launch_pk_body(logn, pk->d_pk, en, sk->d_s, nq, ctx->tab, st);
        CTL_TRY(check_launch());
        CTL_HIP(hipStreamSynchronize(st));
    }
    std::unique_ptr<ctl_evk> evk;
    if (evk_out) {
        evk.reset(new ctl_evk());
        evk->ctx = ctx;
        std::vector<u64> gals;
        for (int r = 0; r < n_rot; ++r) {
            const u64 g = galois_elt(logn, rotations[r]);
            if (g != 1 && std::find(gals.begin(), gals.end(), g) == gals.end()) gals.push_back(g);
        }
        if (relin) gals.push_back(0);
        const size_t key_words = (size_t)nq * 2 * np * n;
        std::vector<u64> hk(key_words);
        std::vector<int64_t> e((size_t)nq * n);
        u64 *en;
        CTL_TRY(slot(ctx, S_DIG, (size_t)nq * np * n, st, &en));
        PrimeList pl{};
        pl.n = np;
        for (int i = 0; i < np; ++i) pl.idx[i] = i;
        for (u64 g : gals) {
            for (int j = 0; j < nq; ++j) {
                Stream sa(seed, TAG_KS_A, g * 64 + (u64)j);
                for (int i = 0; i < np; ++i) {
                    u64 *a = &hk[((size_t)(j * 2 + 1) * np + i) * n];
                    for (int x = 0; x < n; ++x) a[x] = sa.uniform(ctx->hp.mods[i]);
                }
                Stream(seed, TAG_KS_E, g * 64 + (u64)j).gaussian(ctx->hp.cdt, n, &e[(size_t)j * n]);
            }
            u64 *key = static_cast<u64 *>(dev_alloc(ctx, key_words * 8, st));
            if (!key) {
                for (auto &kv : evk->keys) dev_free(ctx, kv.second, st);
                return fail(CTL_ENOMEM, "Galois key allocation failed");
            }
            evk->keys[g] = key;
            CTL_HIP(hipMemcpy(key, hk.data(), key_words * 8, hipMemcpyHostToDevice));
            u64 *stage;
            CTL_TRY(slot(ctx, S_MISC, (size_t)nq * n, st, &stage));
            CTL_HIP(hipMemcpy(stage, e.data(), (size_t)nq * n * 8, hipMemcpyHostToDevice));
            launch_int_ntt(logn, reinterpret_cast<const int64_t *>(stage), en, nq, pl, ctx->tab, st);
            launch_ksk_body(logn, key, en, sk->d_s, g, nq, ctx->tab, st);
            CTL_TRY(check_launch());
            CTL_HIP(hipStreamSynchronize(st));
        }
    }
    if (sk_out) {
        ctx_retain(ctx);
        *sk_out = sk.release();
    } else {
        dev_free(ctx, sk->d_s, st);
    }
    if (pk_out) {
        ctx_retain(ctx);
        *pk_out = pk.release();
    }
    if (evk_out) {
        ctx_retain(ctx);
        *evk_out = evk.release();
    }
    return CTL_OK;
}

int ctl_sk_free(ctl_sk *sk) {
    if (!sk) return CTL_OK;
    ctl_ctx *c = sk->ctx;
    dev_free(c, sk->d_s, nullptr);
    delete sk;
    ctx_release(c);
    return CTL_OK;
}

int ctl_pk_free(ctl_pk *pk) {
    if (!pk) return CTL_OK;
    ctl_ctx *c = pk->ctx;
    dev_free(c, pk->d_pk, nullptr);
    delete pk;
    ctx_release(c);
    return CTL_OK;
}

int ctl_evk_free(ctl_evk *evk) {
    if (!evk) return CTL_OK;
    ctl_ctx *c = evk->ctx;
    for (auto &kv : evk->keys) dev_free(c, kv.second, nullptr);
    delete evk;
    ctx_release(c);
    return CTL_OK;
}

int ctl_sk_export(const ctl_sk *sk, int64_t *coeffs_out) {
    if (!sk || !coeffs_out) return fail(CTL_EINVAL, "null argument");
    std::memcpy(coeffs_out, sk->s.data(), sk->s.size() * 8);
    return CTL_OK;
}

int ctl_pk_export(const ctl_pk *pk, uint64_t *out) {
    if (!pk || !out) return fail(CTL_EINVAL, "null argument");
    CTL_HIP(hipSetDevice(pk->ctx->device));
    CTL_HIP(hipMemcpy(out, pk->d_pk, (size_t)2 * pk->ctx->hp.nq * pk->ctx->hp.n * 8, hipMemcpyDeviceToHost));
    return CTL_OK;
}

int ctl_evk_export(const ctl_evk *evk, uint64_t galois_elt_, uint64_t *out) {
    if (!evk || !out) return fail(CTL_EINVAL, "null argument");
    const u64 *k = find_key(evk, galois_elt_);
    if (!k) return fail(CTL_EKEY, "no key for this Galois element");
    const HostParams &h = evk->ctx->hp;
    CTL_HIP(hipSetDevice(evk->ctx->device));
    CTL_HIP(hipMemcpy(out, k, (size_t)h.nq * 2 * h.np * h.n * 8, hipMemcpyDeviceToHost));
    return CTL_OK;
}

int ctl_evk_galois(const ctl_evk *evk, uint64_t *elts_out, int *n_out) {
    if (!evk || !n_out) return fail(CTL_EINVAL, "null argument");
    int i = 0;
    for (auto &kv : evk->keys) {
        if (elts_out) elts_out[i] = kv.first;
        ++i;
    }
    *n_out = i;
    return CTL_OK;
}


int ctl_ct_packed_bytes(const ctl_params *params, int k, int n_poly, uint64_t *bytes_out) {
    if (!params || !bytes_out || (n_poly != 1 && n_poly != 2)) return fail(CTL_EINVAL, "bad argument");
    HostParams h;
    CTL_TRY(derive_params(params, &h, &g_err));
    if (k < 1 || k > h.nq) return fail(CTL_ELEVEL, "k out of range");
    *bytes_out = packed_bytes(h, k, n_poly);
    return CTL_OK;
}

int ctl_ct_pack(const ctl_params *params, const uint64_t *ct, int k, int n_poly, uint64_t seed, uint8_t *out,
                uint64_t cap, uint64_t *len_out) {
    if (!params || !ct || !out || !len_out || (n_poly != 1 && n_poly != 2)) return fail(CTL_EINVAL, "bad argument");
    HostParams h;
    CTL_TRY(derive_params(params, &h, &g_err));
    if (k < 1 || k > h.nq) return fail(CTL_ELEVEL, "k out of range");
    const u64 len = packed_bytes(h, k, n_poly);
    if (cap < len) return fail(CTL_EINVAL, "output buffer too small");
    const size_t n = h.n;
    for (int p = 0; p < n_poly; ++p)
        for (int i = 0; i < k; ++i)
            for (size_t x = 0; x < n; ++x)
                if (ct[((size_t)p * k + i) * n + x] >= h.mods[i]) return fail(CTL_EINVAL, "word not reduced");
    std::memcpy(out, kMagic, 4);
    out[4] = 1;
    out[5] = (uint8_t)h.logn;
    out[6] = (uint8_t)k;
    out[7] = (uint8_t)n_poly;
    put_u64(out + 8, params_digest(h));
    put_u64(out + 16, n_poly == 1 ? seed : 0);
    uint8_t *w = out + kHeader;
    std::memset(w, 0, len - kHeader);
    u64 bit = 0;
    for (int p = 0; p < n_poly; ++p)
        for (int i = 0; i < k; ++i) {
            const int b = bits_of(h.mods[i]);
            for (size_t x = 0; x < n; ++x, bit += b) {
                const u64 v = ct[((size_t)p * k + i) * n + x];
                for (int j = 0; j < b; ++j)
                    if ((v >> j) & 1) w[(bit + j) >> 3] |= (uint8_t)(1u << ((bit + j) & 7));
            }
        }
    *len_out = len;
    return CTL_OK;
}

int ctl_ct_unpack(const ctl_params *params, const uint8_t *in, uint64_t len, uint64_t *ct_out, int *k_out,
                  int *n_poly_out, uint64_t *seed_out) {
    if (!params || !in || !ct_out || !k_out || !n_poly_out || !seed_out) return fail(CTL_EINVAL, "null argument");
    HostParams h;
    CTL_TRY(derive_params(params, &h, &g_err));
    if (len < (u64)kHeader || std::memcmp(in, kMagic, 4) != 0 || in[4] != 1)
        return fail(CTL_EINVAL, "not a serialized ciphertext of this format");
    const int logn = in[5], k = in[6], n_poly = in[7];
    if (logn != h.logn || get_u64(in + 8) != params_digest(h))
        return fail(CTL_EPARAM, "serialized for another parameter set");
    if (k < 1 || k > h.nq || (n_poly != 1 && n_poly != 2)) return fail(CTL_EINVAL, "bad level or polynomial count");
    if (len != packed_bytes(h, k, n_poly)) return fail(CTL_EINVAL, "length does not match the header");
    const size_t n = h.n;
    std::vector<u64> tmp((size_t)n_poly * k * n);
    const uint8_t *r = in + kHeader;
    u64 bit = 0;
    for (int p = 0; p < n_poly; ++p)
        for (int i = 0; i < k; ++i) {
            const int b = bits_of(h.mods[i]);
            for (size_t x = 0; x < n; ++x, bit += b) {
                u64 v = 0;
                for (int j = 0; j < b; ++j) v |= (u64)((r[(bit + j) >> 3] >> ((bit + j) & 7)) & 1) << j;
                if (v >= h.mods[i]) return fail(CTL_EINVAL, "serialized word not reduced");
                tmp[((size_t)p * k + i) * n + x] = v;
            }
        }
    std::memcpy(ct_out, tmp.data(), tmp.size() * 8);
    *k_out = k;
    *n_poly_out = n_poly;
    *seed_out = get_u64(in + 16);
    return CTL_OK;
}

int ctl_evk_import(ctl_ctx *ctx, const uint64_t *galois_elts, int n_keys, const uint64_t *const *keys,
                   ctl_evk **evk_out) {
    if (!ctx || !evk_out || n_keys < 0 || (n_keys > 0 && (!galois_elts || !keys)))
        return fail(CTL_EINVAL, "bad argument");
    const HostParams &h = ctx->hp;
    const size_t per_prime = (size_t)h.n, key_words = (size_t)h.nq * 2 * h.np * h.n;
    for (int i = 0; i < n_keys; ++i) {
        const u64 g = galois_elts[i];
        if (g != 0 && (g % 2 == 0 || g >= 2 * (u64)h.n || g == 1))
            return fail(CTL_EINVAL, "Galois element " + std::to_string(g) + " is not a rotation of this ring");
        for (int j = 0; j < i; ++j)
            if (galois_elts[j] == g) return fail(CTL_EINVAL, "duplicate Galois element");
        if (!keys[i]) return fail(CTL_EINVAL, "null key array");
        // every word must be a canonical residue of the prime of its row
        for (size_t row = 0; row < (size_t)h.nq * 2 * h.np; ++row) {
            const u64 q = h.mods[row % h.np];
            const uint64_t *w = keys[i] + row * per_prime;
            for (size_t x = 0; x < per_prime; ++x)
                if (w[x] >= q) return fail(CTL_EINVAL, "key word is not reduced modulo its prime");
        }
    }
    CTL_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<ctl_evk> evk(new ctl_evk());
    evk->ctx = ctx;
    for (int i = 0; i < n_keys; ++i) {
        u64 *key = static_cast<u64 *>(dev_alloc(ctx, key_words * 8, nullptr));
        if (!key || hipMemcpy(key, keys[i], key_words * 8, hipMemcpyHostToDevice) != hipSuccess) {
            if (key) dev_free(ctx, key, nullptr);
            for (auto &kv : evk->keys) dev_free(ctx, kv.second, nullptr);
            return fail(key ? CTL_EHIP : CTL_ENOMEM, "Galois key upload failed");
        }
        evk->keys[galois_elts[i]] = key;
    }
    ctx_retain(ctx);
    *evk_out = evk.release();
    return CTL_OK;
}

int ctl_evk_bytes(const ctl_evk *evk, uint64_t *bytes_out) {
    if (!evk || !bytes_out) return fail(CTL_EINVAL, "null argument");
    const HostParams &h = evk->ctx->hp;
    *bytes_out = (uint64_t)evk->keys.size() * h.nq * 2 * h.np * h.n * 8;
    return CTL_OK;
}

int ctl_model_bytes(const ctl_model *m, uint64_t *bytes_out) {
    if (!m || !bytes_out) return fail(CTL_EINVAL, "null argument");
    uint64_t b = 0;
    for (const LayerPlan &L : m->layers) b += (uint64_t)L.nb * bank_rows(L) * m->ctx->hp.n * 8;
    *bytes_out = b;
    return CTL_OK;
}

// ---------------------------------------------------------------- model
int ctl_model_load_ex(ctl_ctx *ctx, const ctl_layer_desc *layers, int n_layers, const double *const *weights,
                      const int64_t *const *pts, const ctl_model_opts *opts, ctl_model **model_out) {
    if ((weights == nullptr) == (pts == nullptr)) return fail(CTL_EINVAL, "give exactly one of weights and pts");
    return make_model(ctx, layers, n_layers, pts, weights, opts, model_out);
}

int ctl_model_load(ctl_ctx *ctx, const ctl_layer_desc *layers, int n_layers, const double *const *weights,
                   ctl_model **model_out) {
    if (!weights) return fail(CTL_EINVAL, "null weights");
    return make_model(ctx, layers, n_layers, nullptr, weights, nullptr, model_out);
}

int ctl_model_load_raw(ctl_ctx *ctx, const ctl_layer_desc *layers, int n_layers, const int64_t *const *pts,
                       ctl_model **model_out) {
    if (!pts) return fail(CTL_EINVAL, "null plaintexts");
    return make_model(ctx, layers, n_layers, pts, nullptr, nullptr, model_out);
}

int ctl_model_free(ctl_model *model) {
    if (!model) return CTL_OK;
    ctl_ctx *c = model->ctx;
    for (u64 *b : model->banks) dev_free(c, b, nullptr);
    delete model;
    ctx_release(c);
    return CTL_OK;
}

int ctl_model_get_info(const ctl_model *m, ctl_model_info *info) {
    if (!m || !info) return fail(CTL_EINVAL, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_layers = (int)m->layers.size();
    info->block = m->block;
    info->items = m->items;
    info->k_in = m->layers[0].k;
    info->k_out = m->k_out;
    info->n_in = m->layers[0].n_in;
    info->n_out = m->layers.back().n_out;
    info->n_rotations = (int)m->rotations.size();
    info->scale_in = m->scale_in;
    info->scale_out = m->scale_out;
    for (size_t l = 0; l < m->layers.size(); ++l) {
        info->layer_k[l] = m->layers[l].k;
        info->layer_t[l] = m->layers[l].t;
    }
    return CTL_OK;
}

int ctl_model_rotations(const ctl_model *m, int32_t *rots_out, int *n_out) {
    if (!m || !n_out) return fail(CTL_EINVAL, "null argument");
    if (rots_out) std::memcpy(rots_out, m->rotations.data(), m->rotations.size() * 4);
    *n_out = (int)m->rotations.size();
    return CTL_OK;
}

// ---------------------------------------------------------------- client encode / encrypt / decrypt
int ctl_encode(ctl_ctx *ctx, const double *slots, double scale, int64_t *coeffs_out) {
    if (!ctx || !slots || !coeffs_out) return fail(CTL_EINVAL, "null argument");
    if (!(scale > 0) || !std::isfinite(scale)) return fail(CTL_ESCALE, "scale must be positive");
    std::vector<int64_t> tmp(ctx->hp.n);
    CTL_TRY(encode_to_int(ctx, slots, scale, tmp.data()));
    std::memcpy(coeffs_out, tmp.data(), tmp.size() * 8);
    return CTL_OK;
}

int ctl_encode_items(ctl_ctx *ctx, const ctl_model *m, const double *x, int items, int64_t *coeffs_out) {
    if (!ctx || !m || !x || !coeffs_out) return fail(CTL_EINVAL, "null argument");
    CTL_SAME(ctx, m, "the model");
    if (items < 1 || items > m->items) return fail(CTL_EINVAL, "items must be in 1..model items");
    const int n_in = m->layers[0].n_in, t = m->layers[0].t;
    std::vector<double> z(ctx->hp.n / 2, 0.0);
    for (int b = 0; b < items; ++b)
        for (int s = 0; s < n_in; ++s) {
            z[(size_t)b * m->block + s] = x[(size_t)b * n_in + s];
            z[(size_t)b * m->block + t + s] = x[(size_t)b * n_in + s];
        }
    return ctl_encode(ctx, z.data(), m->scale_in, coeffs_out);
}

int ctl_encrypt(ctl_ctx *ctx, const ctl_pk *pk, const int64_t *coeffs, uint64_t seed, uint64_t *ct_out, void *stream) {
    if (!ctx || !pk || !coeffs || !ct_out) return fail(CTL_EINVAL, "null argument");
    CTL_SAME(ctx, pk, "the public key");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    const int n = ctx->hp.n, nq = ctx->hp.nq;
    for (int i = 0; i < n; ++i)
        if (coeffs[i] >= (int64_t)(1ull << 62) || coeffs[i] <= -(int64_t)(1ull << 62))
            return fail(CTL_ESCALE, "plaintext coefficient out of range");
    std::vector<int64_t> h((size_t)4 * n);
    Stream(seed, TAG_ENC_V, 0).ternary(n, &h[0]);
    Stream(seed, TAG_ENC_E0, 0).gaussian(ctx->hp.cdt, n, &h[(size_t)n]);
    Stream(seed, TAG_ENC_E1, 0).gaussian(ctx->hp.cdt, n, &h[(size_t)2 * n]);
    std::memcpy(&h[(size_t)3 * n], coeffs, (size_t)n * 8);
    u64 *t4;
    CTL_TRY(slot(ctx, S_COEF2, (size_t)4 * nq * n, st, &t4));
    CTL_TRY(upload_ints(ctx, st, h.data(), 4, nq, t4));
    launch_encrypt(ctx->hp.logn, pk->d_pk, t4, reinterpret_cast<u64 *>(ct_out), nq, ctx->tab, st);
    return check_launch();
}

int ctl_encrypt_sym(ctl_ctx *ctx, const ctl_sk *sk, const int64_t *coeffs, uint64_t seed, uint64_t *ct_out,
                    void *stream) {
    if (!ctx || !sk || !coeffs || !ct_out) return fail(CTL_EINVAL, "null argument");
    CTL_SAME(ctx, sk, "the secret key");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    const int n = ctx->hp.n, nq = ctx->hp.nq;
    std::vector<int64_t> em(n);
    Stream(seed, TAG_SYM_E, 0).gaussian(ctx->hp.cdt, n, em.data());
    for (int i = 0; i < n; ++i) {
        if (coeffs[i] >= (int64_t)(1ull << 62) || coeffs[i] <= -(int64_t)(1ull << 62))
            return fail(CTL_ESCALE, "plaintext coefficient out of range");
        em[i] += coeffs[i];
    }
    std::vector<u64> a;
    seeded_a(ctx, seed, a);
    u64 *emn;
    CTL_TRY(slot(ctx, S_COEF2, (size_t)nq * n, st, &emn));
    CTL_TRY(upload_ints(ctx, st, em.data(), 1, nq, emn));
    u64 *ct = reinterpret_cast<u64 *>(ct_out);
    CTL_HIP(hipMemcpyAsync(ct + (size_t)nq * n, a.data(), (size_t)nq * n * 8, hipMemcpyHostToDevice, st));
    launch_pk_body(ctx->hp.logn, ct, emn, sk->d_s, nq, ctx->tab, st);     // c0 = (e + m) - a s
    CTL_TRY(check_launch());
    CTL_HIP(hipStreamSynchronize(st));
    return CTL_OK;
}

int ctl_expand_seeded(ctl_ctx *ctx, const uint64_t *c0, uint64_t seed, uint64_t *ct_out, void *stream) {
    if (!ctx || !c0 || !ct_out) return fail(CTL_EINVAL, "null argument");
    const int n = ctx->hp.n, nq = ctx->hp.nq;
    for (int i = 0; i < nq; ++i)
        for (int x = 0; x < n; ++x)
            if (c0[(size_t)i * n + x] >= ctx->hp.mods[i]) return fail(CTL_EINVAL, "c0 word not reduced");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    std::vector<u64> a;
    seeded_a(ctx, seed, a);
    u64 *ct = reinterpret_cast<u64 *>(ct_out);
    CTL_HIP(hipMemcpyAsync(ct, c0, (size_t)nq * n * 8, hipMemcpyHostToDevice, st));
    CTL_HIP(hipMemcpyAsync(ct + (size_t)nq * n, a.data(), (size_t)nq * n * 8, hipMemcpyHostToDevice, st));
    CTL_HIP(hipStreamSynchronize(st));
    return CTL_OK;
}

int ctl_decrypt(ctl_ctx *ctx, const ctl_sk *sk, const uint64_t *ct, int k, uint64_t *residues_out, void *stream) {
    if (!ctx || !sk || !ct || !residues_out) return fail(CTL_EINVAL, "null argument");
    CTL_SAME(ctx, sk, "the secret key");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = as_stream(stream);
    const long n = ctx->hp.n;
    u64 *m;
    CTL_TRY(slot(ctx, S_COEF2, (size_t)k * n, st, &m));
    launch_dec_mul(ctx->hp.logn, reinterpret_cast<const u64 *>(ct), sk->d_s, m, k, ctx->tab, st);
    launch_ntt(ctx->hp.logn, true, m, dense_map(k), m, dense_map(k), k, ctx->tab, ctx->knobs, st);
    CTL_TRY(check_launch());
    CTL_HIP(hipMemcpyAsync(residues_out, m, (size_t)k * n * 8, hipMemcpyDeviceToHost, st));
    CTL_HIP(hipStreamSynchronize(st));
    return CTL_OK;
}

int ctl_decode(ctl_ctx *ctx, const uint64_t *residues, int k, double scale, double *slots_out) {
    if (!ctx || !residues || !slots_out) return fail(CTL_EINVAL, "null argument");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    if (!(scale > 0)) return fail(CTL_ESCALE, "scale must be positive");
    const int n = ctx->hp.n;
    std::vector<double> m(n);
    u64 r[kMaxMods];
    for (int x = 0; x < n; ++x) {
        for (int i = 0; i < k; ++i) r[i] = residues[(size_t)i * n + x];
        m[x] = crt_centered_double(r, ctx->hp.mods.data(), k) / scale;
    }
    ctx->enc->decode_real(m.data(), slots_out);
    return CTL_OK;
}

int ctl_decode_items(ctl_ctx *ctx, const ctl_model *m, const uint64_t *residues, double *y_out) {
    if (!ctx || !m || !residues || !y_out) return fail(CTL_EINVAL, "null argument");
    CTL_SAME(ctx, m, "the model");
    std::vector<double> z(ctx->hp.n / 2);
    CTL_TRY(ctl_decode(ctx, residues, m->k_out, m->scale_out, z.data()));
    const LayerPlan &last = m->layers.back();
    const int n_out = last.n_out, off = last.kind == CTL_LAYER_AVGPOOL ? last.f - 1 : 0;
    for (int b = 0; b < m->items; ++b)
        for (int s = 0; s < n_out; ++s) y_out[(size_t)b * n_out + s] = z[(size_t)b * m->block + off + s];
    return CTL_OK;
}

// ---------------------------------------------------------------- server hot path
int ctl_dense(ctl_ctx *ctx, const ctl_model *model, int layer, const ctl_evk *evk, const uint64_t *in,
              uint64_t *out, int n_ct, void *stream) {
    if (!ctx || !model || !evk || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (layer < 0 || layer >= (int)model->layers.size()) return fail(CTL_EINVAL, "layer out of range");
    CTL_SAME(ctx, model, "the model");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    return dense_batch(ctx, as_stream(stream), model, layer, one_key_set(evk, n_ct), n_ct, reinterpret_cast<const u64 *>(in),
                       reinterpret_cast<u64 *>(out));
}

int ctl_dense_groups(ctl_ctx *ctx, const ctl_model *const *models, const int *counts, int n_groups, int layer,
                     const ctl_evk *evk, const uint64_t *in, uint64_t *out, void *stream) {
    if (!ctx || !models || !counts || !evk || !in || !out || n_groups < 1 || n_groups > 4096)
        return fail(CTL_EINVAL, "bad argument");
    CTL_SAME(ctx, evk, "the evaluation key set");
    int n_ct = 0, k = -1;
    for (int g = 0; g < n_groups; ++g) {
        const ctl_model *m = models[g];
        if (!m) return fail(CTL_EINVAL, "null model");
        CTL_SAME(ctx, m, "every model");
        if (counts[g] < 1) return fail(CTL_EINVAL, "every group needs at least one ciphertext");
        if (layer < 0 || layer >= (int)m->layers.size()) return fail(CTL_EINVAL, "layer out of range");
        const LayerPlan &L = m->layers[layer];
        if (!L.qp) return fail(CTL_EINVAL, "every layer must keep its baby steps over Q*P (CTL_LAYER_BABY_QP)");
        if (k >= 0 && L.k != k) return fail(CTL_ELEVEL, "every group's layer must start at the same level");
        k = L.k;
        if (L.t1 - 1 > kMaxKeysPerLaunch || L.t2 - 1 > kMaxKeysPerLaunch)
            return fail(CTL_EINVAL, "t1 and t2 must be at most 65");
        for (long r : L.rots1)
            CTL_TRY(need_key(one_key_set(evk, 1), galois_elt(ctx->hp.logn, r), "Galois key for rotation " + std::to_string(r)));
        for (int k2 = 1; k2 < L.t2; ++k2)
            CTL_TRY(need_key(one_key_set(evk, 1), galois_elt(ctx->hp.logn, (long)k2 * L.t1),
                             "Galois key for rotation " + std::to_string(k2 * L.t1)));
        n_ct += counts[g];
    }
    CTL_HIP(hipSetDevice(ctx->device));
    return dense_qp_groups(ctx, as_stream(stream), models, counts, n_groups, layer, one_key_set(evk, n_ct),
                           reinterpret_cast<const u64 *>(in), reinterpret_cast<u64 *>(out));
}

int ctl_square(ctl_ctx *ctx, const ctl_evk *evk, int k, const uint64_t *in, uint64_t *out, int n_ct, void *stream) {
    if (!ctx || !evk || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 2 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    return square_batch(ctx, as_stream(stream), one_key_set(evk, n_ct), k, n_ct, reinterpret_cast<const u64 *>(in),
                        reinterpret_cast<u64 *>(out));
}

// Scratch words of square_batch for B ciphertexts at k primes: tensor 3k, relinearized 2k (ModDown
// and rescale apart), coefficient-form digits k, ModUp digits k(k+1), key product 2(k+1), ModDown
// P rows 2, rescale rows 2 (each times N, per ciphertext; every size is a multiple of the 32-word
// carve alignment; ModDown and rescale as one pass take 4 coefficient rows and no relinearized
// rows, within this bound).
static size_t square_scratch_words(int k, long n, int B) { return (size_t)B * n * ((size_t)k * k + 9 * k + 6); }

int ctl_square_noalloc(ctl_ctx *ctx, const ctl_evk *evk, int k, const uint64_t *in, uint64_t *out, int n_ct,
                       void *stream) {
    if (!ctx || !evk || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 2 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_SAME(ctx, evk, "the evaluation key set");
    if (!ctx->scratch) return fail(CTL_EHIP, "no scratch array on this device");
    if (square_scratch_words(k, ctx->hp.n, n_ct) > kScratchWords)
        return fail(CTL_EINVAL, "batch needs " + std::to_string(square_scratch_words(k, ctx->hp.n, n_ct) * 8) +
                                    " bytes of scratch; the fixed array holds " +
                                    std::to_string((unsigned long long)CTL_NOALLOC_SCRATCH_BYTES));
    CTL_HIP(hipSetDevice(ctx->device));
    struct Arena {                               // carve from the scratch array for this call only
        ctl_ctx *c;
        explicit Arena(ctl_ctx *c_) : c(c_) { c->arena = true; c->arena_used = 0; }
        ~Arena() { c->arena = false; c->arena_used = 0; }
    } arena(ctx);
    return square_batch(ctx, as_stream(stream), one_key_set(evk, n_ct), k, n_ct, reinterpret_cast<const u64 *>(in),
                        reinterpret_cast<u64 *>(out));
}

int ctl_replicate(ctl_ctx *ctx, const ctl_evk *evk, int k, int width, const uint64_t *in, uint64_t *out,
                  int n_ct, void *stream) {
    if (!ctx || !evk || !in || !out || n_ct < 1 || width < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    return replicate_batch(ctx, as_stream(stream), one_key_set(evk, n_ct), k, n_ct, width, reinterpret_cast<const u64 *>(in),
                           reinterpret_cast<u64 *>(out));
}

int ctl_rotate(ctl_ctx *ctx, const ctl_evk *evk, int k, int rotation, const uint64_t *in, uint64_t *out,
               int n_ct, void *stream) {
    if (!ctx || !evk || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 1 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    return rotate_batch(ctx, as_stream(stream), one_key_set(evk, n_ct), k, n_ct, rotation, reinterpret_cast<const u64 *>(in),
                        reinterpret_cast<u64 *>(out));
}

int ctl_rescale(ctl_ctx *ctx, int k, const uint64_t *in, uint64_t *out, int n_ct, void *stream) {
    if (!ctx || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 2 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_HIP(hipSetDevice(ctx->device));
    return rescale_batch(ctx, as_stream(stream), k, n_ct, reinterpret_cast<const u64 *>(in),
                         reinterpret_cast<u64 *>(out));
}

int ctl_forward(ctl_ctx *ctx, const ctl_model *m, const ctl_evk *evk, const uint64_t *in, uint64_t *out,
                int n_ct, void *stream) {
    if (!ctx || !m || !evk || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    CTL_SAME(ctx, m, "the model");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    return forward_batch(ctx, as_stream(stream), m, one_key_set(evk, n_ct), n_ct, reinterpret_cast<const u64 *>(in),
                         reinterpret_cast<u64 *>(out));
}

int ctl_forward_multi(ctl_ctx *ctx, const ctl_model *m, const ctl_evk *const *evks, const uint64_t *in,
                      uint64_t *out, int n_ct, void *stream) {
    if (!ctx || !m || !evks || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    CTL_SAME(ctx, m, "the model");
    KeySet ks;
    for (int b = 0; b < n_ct; ++b) {
        if (!evks[b]) return fail(CTL_EINVAL, "null evaluation key set");
        CTL_SAME(ctx, evks[b], "every evaluation key set");
        if (!ks.runs.empty() && ks.runs.back().evk == evks[b])
            ++ks.runs.back().nb;
        else
            ks.runs.push_back({evks[b], b, 1});
    }
    CTL_HIP(hipSetDevice(ctx->device));
    return forward_batch(ctx, as_stream(stream), m, ks, n_ct, reinterpret_cast<const u64 *>(in),
                         reinterpret_cast<u64 *>(out));
}

int ctl_mul(ctl_ctx *ctx, const ctl_evk *evk, int k, const uint64_t *a, const uint64_t *b, uint64_t *out,
            int n_ct, void *stream) {
    if (!ctx || !evk || !a || !b || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 2 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    return mul_batch(ctx, as_stream(stream), one_key_set(evk, n_ct), k, n_ct, reinterpret_cast<const u64 *>(a),
                     reinterpret_cast<const u64 *>(b), reinterpret_cast<u64 *>(out));
}

int ctl_poly3(ctl_ctx *ctx, const ctl_evk *evk, int k, double scale, const double *coef, const uint64_t *in,
              uint64_t *out, int n_ct, void *stream, double *scale_out) {
    if (!ctx || !evk || !coef || !in || !out || n_ct < 1) return fail(CTL_EINVAL, "bad argument");
    if (k < 3 || k > ctx->hp.nq) return fail(CTL_ELEVEL, "k out of range");
    if (!(scale > 0) || !std::isfinite(scale)) return fail(CTL_ESCALE, "scale must be positive");
    CTL_SAME(ctx, evk, "the evaluation key set");
    CTL_HIP(hipSetDevice(ctx->device));
    CTL_TRY(poly3_batch(ctx, as_stream(stream), one_key_set(evk, n_ct), k, n_ct, scale, coef, reinterpret_cast<const u64 *>(in),
                        reinterpret_cast<u64 *>(out)));
    if (scale_out) {
        int64_t C[4];
        *scale_out = poly3_consts(ctx, k, scale, coef, C);
    }
    return CTL_OK;
}

}  // extern "C"
