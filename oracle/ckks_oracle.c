/*
 * Plain CPU oracle of RNS-CKKS for the encrypted frozen-layer forward pass.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load this library. The GPU library never links, includes or calls it, and this file
 * uses nothing from the GPU library.
 *
 * Everything here is written for obviousness, not speed: scalar loops, 128-bit products reduced
 * with the % operator, one residue polynomial at a time.
 *
 * The paper (CryptoTL, Section 3.1) fixes only the circuit level: CKKS with scale Delta and
 * rescaling after multiplications ("The CKKS HE scheme"), SIMD slots with cyclic left rotations
 * ("SIMD Encoding"), the baby-step giant-step diagonal dense layer (Eq. (1), "Dense-Layer"),
 * slot packing of several items ("Multiple Predictions") and the prime chain ("Multiplicative
 * Depth"). Everything below the CKKS-operation level is a reading this code takes explicitly:
 *
 *   primes      largest prime below 2^b with q = 1 (mod 2N), listed order, distinct, P last
 *   psi         smallest primitive 2N-th root of unity mod q
 *   NTT         NTT(a)[i] = sum_k a_k psi^{(2 brv(i) + 1) k}  (bit-reversed evaluation order)
 *   slots       slot j <-> zeta^{5^j}; left rotation by r <-> Galois element 5^r mod 2N
 *   sampling    ChaCha20 (RFC 8439) keyed by the seed; ternary secret; discrete Gaussian by an
 *               FP64 cumulative table; uniform residues by rejection
 *   keys        one-prime digits (one digit per ciphertext prime), one special prime P
 *   rounding    ModDown and rescale round to nearest through centered residues
 *
 * Parity pins (checked by the CPU tests against independent definitions): primes by trial
 * properties, NTT against the O(N^2) definition and negacyclic schoolbook products, automorphism
 * composition laws, ModDown/rescale against big-integer round(x/P), ChaCha20 against the RFC 8439
 * block test vector, decrypt(encrypt(m)) against m within the noise bound, hoisted rotations
 * against unhoisted ones, the BSGS dense layer against an FP64 matrix product, its Q*P baby-step
 * variant against the single-ModDown one where they coincide (t1 = 1) and against plain
 * rotations when a unit plaintext selects one baby step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

#define OR_MAXP 20          /* ciphertext primes + special prime */
#define OR_CDT_N 39         /* Gaussian support -19..19 */
#define OR_TAIL 19

/* ---------------------------------------------------------------- scalar modular arithmetic */

static u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
/* a, b < q < 2^62 throughout, so the sums below cannot overflow. */
static u64 addm(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
static u64 negm(u64 a, u64 q) { return a == 0 ? 0 : q - a; }

static u64 powm(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulm(r, a, q);
        a = mulm(a, a, q);
        e >>= 1;
    }
    return r;
}

static u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); } /* q prime */

/* Deterministic Miller-Rabin: the first twelve prime bases decide every n < 2^64. */
static int is_prime(u64 n) {
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; r++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powm(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int k = 1; k < r; k++) {
            x = mulm(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

static u32 brv(u32 x, int bits) {
    u32 r = 0;
    for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* Centered lift: x in [0, qf) read as the representative in (-qf/2, qf/2), reduced mod qt. */
static u64 lift_centered(u64 x, u64 qf, u64 qt) {
    if (x > (qf - 1) / 2) return subm(x % qt, qf % qt, qt);
    return x % qt;
}

/* ---------------------------------------------------------------- context */

typedef struct {
    int logn, n;
    int nq;                 /* ciphertext primes q_0..q_{nq-1} */
    int np;                 /* nq + 1: index nq is the special prime P */
    u64 q[OR_MAXP];
    u64 psi[OR_MAXP];
    u64 *fw[OR_MAXP];       /* fw[i][m] = psi_i^{brv(m)} */
    u64 *iw[OR_MAXP];       /* iw[i][m] = psi_i^{-brv(m)} */
    u64 ninv[OR_MAXP];
    double sigma;
    u64 cdt[OR_CDT_N];
} or_ctx;

/* Prime selection: for each requested bit size b (ciphertext primes in listed order, then P),
 * scan 2^b - 2N + 1, 2^b - 4N + 1, ... downward and take the first prime not already taken. */
int or_find_primes(int logn, const int *bits, int count, u64 *out) {
    u64 two_n = 2ull << logn;
    for (int i = 0; i < count; i++) {
        if (bits[i] < logn + 2 || bits[i] > 61) return -1;
        u64 c = (1ull << bits[i]) - two_n + 1;
        for (;;) {
            int used = 0;
            for (int j = 0; j < i; j++) used |= (out[j] == c);
            if (!used && is_prime(c)) break;
            if (c < two_n + 1) return -7;
            c -= two_n;
        }
        out[i] = c;
    }
    return 0;
}

/* Smallest primitive 2N-th root of unity mod q. */
u64 or_min_psi(u64 q, int logn) {
    u64 n = 1ull << logn, two_n = 2 * n;
    u64 w = 0;
    for (u64 g = 2; g < q; g++) {
        w = powm(g, (q - 1) / two_n, q);
        if (powm(w, n, q) == q - 1) break;   /* order exactly 2N */
    }
    u64 best = w, w2 = mulm(w, w, q), cur = w;
    for (u64 k = 1; k < two_n; k += 2) {     /* every odd power is again primitive */
        if (cur < best) best = cur;
        cur = mulm(cur, w2, q);
    }
    return best;
}

static void build_cdt(or_ctx *c) {
    /* rho(e) = exp(-e^2 / (2 sigma^2)) on e = -19..19; T[m] = floor(2^53 * C[m]) where C[m] is
     * the running sum over e = -19..-19+m (added in increasing e) divided by the total. */
    double rho[OR_CDT_N], total = 0.0, run = 0.0;
    for (int m = 0; m < OR_CDT_N; m++) {
        double e = (double)(m - OR_TAIL);
        rho[m] = exp(-(e * e) / (2.0 * c->sigma * c->sigma));
    }
    for (int m = 0; m < OR_CDT_N; m++) total += rho[m];
    for (int m = 0; m < OR_CDT_N; m++) {
        run += rho[m];
        c->cdt[m] = (u64)ldexp(run / total, 53);
    }
    c->cdt[OR_CDT_N - 1] = 1ull << 53;
}

or_ctx *or_ctx_new(int logn, int nq, const int *q_bits, int p_bits, double sigma) {
    if (nq < 1 || nq + 1 > OR_MAXP || logn < 2 || logn > 17) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->logn = logn;
    c->n = 1 << logn;
    c->nq = nq;
    c->np = nq + 1;
    c->sigma = sigma;
    int bits[OR_MAXP];
    for (int i = 0; i < nq; i++) bits[i] = q_bits[i];
    bits[nq] = p_bits;
    if (or_find_primes(logn, bits, c->np, c->q) != 0) { free(c); return NULL; }
    for (int i = 0; i < c->np; i++) {
        u64 q = c->q[i];
        c->psi[i] = or_min_psi(q, logn);
        u64 pinv = invm(c->psi[i], q);
        c->fw[i] = (u64 *)malloc(sizeof(u64) * c->n);
        c->iw[i] = (u64 *)malloc(sizeof(u64) * c->n);
        for (int m = 0; m < c->n; m++) {
            u32 e = brv((u32)m, logn);
            c->fw[i][m] = powm(c->psi[i], e, q);
            c->iw[i][m] = powm(pinv, e, q);
        }
        c->ninv[i] = invm((u64)c->n % q, q);
    }
    build_cdt(c);
    return c;
}

void or_ctx_free(or_ctx *c) {
    if (!c) return;
    for (int i = 0; i < c->np; i++) { free(c->fw[i]); free(c->iw[i]); }
    free(c);
}

int or_ctx_n(const or_ctx *c) { return c->n; }
int or_ctx_nq(const or_ctx *c) { return c->nq; }
void or_ctx_primes(const or_ctx *c, u64 *out) { for (int i = 0; i < c->np; i++) out[i] = c->q[i]; }
void or_ctx_psis(const or_ctx *c, u64 *out) { for (int i = 0; i < c->np; i++) out[i] = c->psi[i]; }
void or_ctx_cdt(const or_ctx *c, u64 *out) { for (int i = 0; i < OR_CDT_N; i++) out[i] = c->cdt[i]; }

/* ---------------------------------------------------------------- NTT on one residue */

/* Forward negacyclic NTT in place (Cooley-Tukey butterflies, natural order in, bit-reversed
 * order out): afterwards a[i] = sum_k a_k psi^{(2 brv(i) + 1) k}. */
static void ntt_fwd(const or_ctx *c, int pi, u64 *a) {
    u64 q = c->q[pi];
    int n = c->n, t = n;
    for (int m = 1; m < n; m <<= 1) {
        t >>= 1;
        for (int i = 0; i < m; i++) {
            u64 w = c->fw[pi][m + i];
            int j1 = 2 * i * t;
            for (int j = j1; j < j1 + t; j++) {
                u64 u = a[j], v = mulm(a[j + t], w, q);
                a[j] = addm(u, v, q);
                a[j + t] = subm(u, v, q);
            }
        }
    }
}

/* Inverse of ntt_fwd (Gentleman-Sande butterflies, bit-reversed in, natural out, times N^-1). */
static void ntt_inv(const or_ctx *c, int pi, u64 *a) {
    u64 q = c->q[pi];
    int n = c->n, t = 1;
    for (int m = n; m > 1; m >>= 1) {
        int h = m >> 1, j1 = 0;
        for (int i = 0; i < h; i++) {
            u64 w = c->iw[pi][h + i];
            for (int j = j1; j < j1 + t; j++) {
                u64 u = a[j], v = a[j + t];
                a[j] = addm(u, v, q);
                a[j + t] = mulm(subm(u, v, q), w, q);
            }
            j1 += 2 * t;
        }
        t <<= 1;
    }
    for (int j = 0; j < n; j++) a[j] = mulm(a[j], c->ninv[pi], q);
}

void or_ntt(const or_ctx *c, int pi, u64 *a, int inverse) {
    if (inverse) ntt_inv(c, pi, a);
    else ntt_fwd(c, pi, a);
}

/* ---------------------------------------------------------------- automorphisms */

/* Coefficient form: a_k X^k -> a_k X^{g k mod 2N}, negated when g k mod 2N >= N. */
void or_automorph_coef(const or_ctx *c, int pi, u64 g, const u64 *in, u64 *out) {
    u64 two_n = 2ull * c->n, q = c->q[pi];
    for (int k = 0; k < c->n; k++) {
        u64 e = (g * (u64)k) % two_n;
        if (e < (u64)c->n) out[e] = in[k];
        else out[e - c->n] = negm(in[k], q);
    }
}

/* NTT form: slot i holds a(psi^{2 brv(i)+1}); sigma_g(a) there equals a(psi^{g (2 brv(i)+1)}),
 * which is stored at index brv((g (2 brv(i)+1) mod 2N - 1) / 2). A pure permutation. */
void or_automorph_ntt(const or_ctx *c, u64 g, const u64 *in, u64 *out) {
    u64 two_n = 2ull * c->n;
    for (int i = 0; i < c->n; i++) {
        u64 e = (g * (2ull * brv((u32)i, c->logn) + 1)) % two_n;
        out[i] = in[brv((u32)((e - 1) / 2), c->logn)];
    }
}

/* Galois element of a left rotation by r slots: 5^(r mod N/2) mod 2N. */
u64 or_galois_elt(const or_ctx *c, long r) {
    long half = c->n / 2;
    long e = ((r % half) + half) % half;
    u64 g = 1, two_n = 2ull * c->n;
    for (long i = 0; i < e; i++) g = (g * 5) % two_n;
    return g;
}

/* ---------------------------------------------------------------- ChaCha20 (RFC 8439) */

#define ROTL32(v, s) (((v) << (s)) | ((v) >> (32 - (s))))
#define QR(a, b, c, d)                                      \
    a += b; d ^= a; d = ROTL32(d, 16);                      \
    c += d; b ^= c; b = ROTL32(b, 12);                      \
    a += b; d ^= a; d = ROTL32(d, 8);                       \
    c += d; b ^= c; b = ROTL32(b, 7);

/* One 64-byte block: key (8 words), block counter, nonce (3 words). */
void or_chacha20_block(const u32 *key, u32 counter, const u32 *nonce, uint8_t *out) {
    u32 s[16], x[16];
    s[0] = 0x61707865u; s[1] = 0x3320646eu; s[2] = 0x79622d32u; s[3] = 0x6b206574u;
    for (int i = 0; i < 8; i++) s[4 + i] = key[i];
    s[12] = counter;
    s[13] = nonce[0]; s[14] = nonce[1]; s[15] = nonce[2];
    memcpy(x, s, sizeof(s));
    for (int r = 0; r < 10; r++) {
        QR(x[0], x[4], x[8], x[12]);
        QR(x[1], x[5], x[9], x[13]);
        QR(x[2], x[6], x[10], x[14]);
        QR(x[3], x[7], x[11], x[15]);
        QR(x[0], x[5], x[10], x[15]);
        QR(x[1], x[6], x[11], x[12]);
        QR(x[2], x[7], x[8], x[13]);
        QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; i++) {
        u32 v = x[i] + s[i];
        out[4 * i + 0] = (uint8_t)(v);
        out[4 * i + 1] = (uint8_t)(v >> 8);
        out[4 * i + 2] = (uint8_t)(v >> 16);
        out[4 * i + 3] = (uint8_t)(v >> 24);
    }
}

/* A byte stream: key = the 64-bit seed little-endian, zero-padded to 32 bytes;
 * nonce = (purpose tag, low 32 bits of index, high 32 bits of index); counter from 0. */
typedef struct {
    u32 key[8], nonce[3], counter;
    uint8_t buf[64];
    int pos;
} stream_t;

static void stream_init(stream_t *st, u64 seed, u32 tag, u64 index) {
    memset(st, 0, sizeof(*st));
    st->key[0] = (u32)seed;
    st->key[1] = (u32)(seed >> 32);
    st->nonce[0] = tag;
    st->nonce[1] = (u32)index;
    st->nonce[2] = (u32)(index >> 32);
    st->pos = 64;
}

static uint8_t stream_u8(stream_t *st) {
    if (st->pos == 64) {
        or_chacha20_block(st->key, st->counter++, st->nonce, st->buf);
        st->pos = 0;
    }
    return st->buf[st->pos++];
}

static u64 stream_u64(stream_t *st) {
    u64 v = 0;
    for (int i = 0; i < 8; i++) v |= (u64)stream_u8(st) << (8 * i);
    return v;
}

enum { TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_KS_A = 4, TAG_KS_E = 5,
       TAG_ENC_V = 8, TAG_ENC_E0 = 9, TAG_ENC_E1 = 10, TAG_SYM_A = 11, TAG_SYM_E = 12 };

static void sample_ternary(stream_t *st, int n, int64_t *out) {
    for (int k = 0; k < n; k++) {
        uint8_t b;
        do { b = stream_u8(st); } while (b == 255);
        out[k] = (int64_t)(b % 3) - 1;
    }
}

static void sample_gauss(const or_ctx *c, stream_t *st, int n, int64_t *out) {
    for (int k = 0; k < n; k++) {
        u64 u = stream_u64(st) >> 11;
        int m = 0;
        while (u >= c->cdt[m]) m++;
        out[k] = (int64_t)m - OR_TAIL;
    }
}

static u64 sample_uniform1(stream_t *st, u64 q) {
    u64 lim = (u64)((((u128)1) << 64) / q * q);
    u64 x;
    do { x = stream_u64(st); } while (x >= lim);
    return x % q;
}

/* Test hook: kind 0 ternary, 1 Gaussian, 2 uniform mod `modulus` (all as int64/u64 words). */
void or_sample(const or_ctx *c, u64 seed, u32 tag, u64 index, int kind, u64 modulus, int n,
               int64_t *out) {
    stream_t st;
    stream_init(&st, seed, tag, index);
    if (kind == 0) sample_ternary(&st, n, out);
    else if (kind == 1) sample_gauss(c, &st, n, out);
    else for (int k = 0; k < n; k++) out[k] = (int64_t)sample_uniform1(&st, modulus);
}

/* ---------------------------------------------------------------- polynomial helpers */

/* Signed small coefficients -> NTT-form residue mod prime pi. */
static void small_to_ntt(const or_ctx *c, int pi, const int64_t *s, u64 *out) {
    u64 q = c->q[pi];
    for (int k = 0; k < c->n; k++) {
        int64_t v = s[k] % (int64_t)q;
        out[k] = v < 0 ? (u64)(v + (int64_t)q) : (u64)v;
    }
    ntt_fwd(c, pi, out);
}

/* Prime index of residue slot i in a buffer that holds k ciphertext primes then P. */
static int ext_prime(int k, int i, const or_ctx *c) { return i < k ? i : c->nq; }

/* ---------------------------------------------------------------- keys */

/* Secret key: ternary coefficients s (int64[N]). */
void or_keygen_secret(const or_ctx *c, u64 seed, int64_t *s) {
    stream_t st;
    stream_init(&st, seed, TAG_SK, 0);
    sample_ternary(&st, c->n, s);
}

/* s in NTT form for all np primes: [np][N]. */
void or_secret_ntt(const or_ctx *c, const int64_t *s, u64 *s_ntt) {
    for (int i = 0; i < c->np; i++) small_to_ntt(c, i, s, s_ntt + (size_t)i * c->n);
}

/* Public key pk = (b, a) over q_0..q_L, [2][nq][N] NTT form: a uniform (drawn directly as NTT
 * values, prime by prime), e Gaussian, b = -a s + e. */
void or_keygen_public(const or_ctx *c, u64 seed, const int64_t *s, u64 *pk) {
    int n = c->n, nq = c->nq;
    u64 *sn = (u64 *)malloc(sizeof(u64) * n), *en = (u64 *)malloc(sizeof(u64) * n);
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * n);
    stream_t sa, se;
    stream_init(&sa, seed, TAG_PK_A, 0);
    stream_init(&se, seed, TAG_PK_E, 0);
    sample_gauss(c, &se, n, e);
    for (int i = 0; i < nq; i++) {
        u64 q = c->q[i];
        u64 *b = pk + (size_t)i * n, *a = pk + (size_t)(nq + i) * n;
        for (int k = 0; k < n; k++) a[k] = sample_uniform1(&sa, q);
        small_to_ntt(c, i, s, sn);
        small_to_ntt(c, i, e, en);
        for (int k = 0; k < n; k++) b[k] = addm(negm(mulm(a[k], sn[k], q), q), en[k], q);
    }
    free(sn); free(en); free(e);
}

/* Key-switching key from s' (given in NTT form over the nq ciphertext primes) to s.
 * Layout [nq digits][2][np][N], NTT form. For digit j and prime i:
 *   b_j = -a_j s + e_j + (i == j ? [P]_{q_i} s' : 0)  (mod q_i),   b_j = -a_j s + e_j  (mod P).
 * The draws use index = g * 64 + j, with g the Galois element (0 for relinearization). */
static void keygen_switch(const or_ctx *c, u64 seed, u64 g, const int64_t *s, const u64 *sp_ntt,
                          u64 *key) {
    int n = c->n, nq = c->nq, np = c->np;
    u64 P = c->q[nq];
    u64 *sn = (u64 *)malloc(sizeof(u64) * (size_t)np * n), *en = (u64 *)malloc(sizeof(u64) * n);
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int i = 0; i < np; i++) small_to_ntt(c, i, s, sn + (size_t)i * n);
    for (int j = 0; j < nq; j++) {
        stream_t sa, se;
        stream_init(&sa, seed, TAG_KS_A, g * 64 + (u64)j);
        stream_init(&se, seed, TAG_KS_E, g * 64 + (u64)j);
        sample_gauss(c, &se, n, e);
        for (int i = 0; i < np; i++) {
            u64 q = c->q[i];
            u64 *b = key + ((size_t)(j * 2 + 0) * np + i) * n;
            u64 *a = key + ((size_t)(j * 2 + 1) * np + i) * n;
            const u64 *si = sn + (size_t)i * n;
            for (int k = 0; k < n; k++) a[k] = sample_uniform1(&sa, q);
            small_to_ntt(c, i, e, en);
            for (int k = 0; k < n; k++) b[k] = addm(negm(mulm(a[k], si[k], q), q), en[k], q);
            if (i == j) {
                u64 pm = P % q;
                const u64 *spi = sp_ntt + (size_t)i * n;
                for (int k = 0; k < n; k++) b[k] = addm(b[k], mulm(pm, spi[k], q), q);
            }
        }
    }
    free(sn); free(en); free(e);
}

/* Galois key for element g: switches from sigma_g(s) to s. */
void or_keygen_galois(const or_ctx *c, u64 seed, const int64_t *s, u64 g, u64 *key) {
    int n = c->n, nq = c->nq;
    u64 *sp = (u64 *)malloc(sizeof(u64) * (size_t)nq * n);
    u64 *tmp = (u64 *)malloc(sizeof(u64) * n);
    for (int i = 0; i < nq; i++) {
        u64 q = c->q[i];
        for (int k = 0; k < n; k++) {
            int64_t v = s[k];
            tmp[k] = v < 0 ? q - 1 : (u64)v;
        }
        or_automorph_coef(c, i, g, tmp, sp + (size_t)i * n);
        ntt_fwd(c, i, sp + (size_t)i * n);
    }
    keygen_switch(c, seed, g, s, sp, key);
    free(sp); free(tmp);
}

/* Relinearization key: switches from s^2 to s. */
void or_keygen_relin(const or_ctx *c, u64 seed, const int64_t *s, u64 *key) {
    int n = c->n, nq = c->nq;
    u64 *sp = (u64 *)malloc(sizeof(u64) * (size_t)nq * n);
    for (int i = 0; i < nq; i++) {
        u64 *r = sp + (size_t)i * n;
        small_to_ntt(c, i, s, r);
        for (int k = 0; k < n; k++) r[k] = mulm(r[k], r[k], c->q[i]);
    }
    keygen_switch(c, seed, 0, s, sp, key);
    free(sp);
}

/* ---------------------------------------------------------------- encrypt / decrypt */

/* Plaintext from signed integer coefficients: [k][N] NTT form over q_0..q_{k-1}. */
void or_plaintext(const or_ctx *c, const int64_t *m, int k, u64 *pt) {
    for (int i = 0; i < k; i++) small_to_ntt(c, i, m, pt + (size_t)i * c->n);
}

/* The same plaintext over q_0..q_{k-1}, P: [k+1][N], row k under the special prime. */
void or_plaintext_ext(const or_ctx *c, const int64_t *m, int k, u64 *pt) {
    or_plaintext(c, m, k, pt);
    small_to_ntt(c, c->nq, m, pt + (size_t)k * c->n);
}

/* Public-key encryption at the top level: ct = (v b + e0 + m, v a + e1), [2][nq][N]. */
void or_encrypt(const or_ctx *c, const u64 *pk, const int64_t *m, u64 seed, u64 *ct) {
    int n = c->n, nq = c->nq;
    int64_t *v = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *e0 = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *e1 = (int64_t *)malloc(sizeof(int64_t) * n);
    u64 *vn = (u64 *)malloc(sizeof(u64) * n), *tn = (u64 *)malloc(sizeof(u64) * n);
    stream_t sv, s0, s1;
    stream_init(&sv, seed, TAG_ENC_V, 0);
    stream_init(&s0, seed, TAG_ENC_E0, 0);
    stream_init(&s1, seed, TAG_ENC_E1, 0);
    sample_ternary(&sv, n, v);
    sample_gauss(c, &s0, n, e0);
    sample_gauss(c, &s1, n, e1);
    for (int i = 0; i < nq; i++) {
        u64 q = c->q[i];
        const u64 *b = pk + (size_t)i * n, *a = pk + (size_t)(nq + i) * n;
        u64 *c0 = ct + (size_t)i * n, *c1 = ct + (size_t)(nq + i) * n;
        small_to_ntt(c, i, v, vn);
        small_to_ntt(c, i, m, tn);
        for (int k = 0; k < n; k++) c0[k] = addm(mulm(vn[k], b[k], q), tn[k], q);
        small_to_ntt(c, i, e0, tn);
        for (int k = 0; k < n; k++) c0[k] = addm(c0[k], tn[k], q);
        small_to_ntt(c, i, e1, tn);
        for (int k = 0; k < n; k++) c1[k] = addm(mulm(vn[k], a[k], q), tn[k], q);
    }
    free(v); free(e0); free(e1); free(vn); free(tn);
}

/* Decrypt a [2][k][N] ciphertext: coefficient-form residues of c0 + c1 s, [k][N]. */
void or_decrypt(const or_ctx *c, const int64_t *s, const u64 *ct, int k, u64 *out) {
    int n = c->n;
    u64 *sn = (u64 *)malloc(sizeof(u64) * n);
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        const u64 *c0 = ct + (size_t)i * n, *c1 = ct + (size_t)(k + i) * n;
        u64 *o = out + (size_t)i * n;
        small_to_ntt(c, i, s, sn);
        for (int j = 0; j < n; j++) o[j] = addm(c0[j], mulm(c1[j], sn[j], q), q);
        ntt_inv(c, i, o);
    }
    free(sn);
}

/* ---------------------------------------------------------------- key switching */

/* ModUp: d = [k][N] NTT form over q_0..q_{k-1}. Digit j is the centered lift of d_j (coefficient
 * form) to every prime of q_0..q_{k-1}, P; output [k digits][k+1][N] NTT form. */
void or_modup(const or_ctx *c, int k, const u64 *d, u64 *digits) {
    int n = c->n;
    u64 *coef = (u64 *)malloc(sizeof(u64) * n);
    for (int j = 0; j < k; j++) {
        memcpy(coef, d + (size_t)j * n, sizeof(u64) * n);
        ntt_inv(c, j, coef);
        for (int t = 0; t <= k; t++) {
            int pt = ext_prime(k, t, c);
            u64 *o = digits + ((size_t)j * (k + 1) + t) * n;
            if (t == j) { memcpy(o, d + (size_t)j * n, sizeof(u64) * n); continue; }
            for (int x = 0; x < n; x++) o[x] = lift_centered(coef[x], c->q[j], c->q[pt]);
            ntt_fwd(c, pt, o);
        }
    }
    free(coef);
}

/* Inner product of ModUp digits with a key restricted to level k-1: u = sum_j D_j (b_j, a_j),
 * output [2][k+1][N] over q_0..q_{k-1}, P. Optionally applies sigma_g to each digit first. */
static void key_inner(const or_ctx *c, int k, const u64 *digits, const u64 *key, u64 g, u64 *u) {
    int n = c->n, np = c->np;
    u64 *tmp = (u64 *)malloc(sizeof(u64) * n);
    memset(u, 0, sizeof(u64) * 2 * (k + 1) * n);
    for (int j = 0; j < k; j++) {
        for (int t = 0; t <= k; t++) {
            int pt = ext_prime(k, t, c);
            u64 q = c->q[pt];
            const u64 *dj = digits + ((size_t)j * (k + 1) + t) * n;
            if (g != 1) { or_automorph_ntt(c, g, dj, tmp); dj = tmp; }
            const u64 *b = key + ((size_t)(j * 2 + 0) * np + pt) * n;
            const u64 *a = key + ((size_t)(j * 2 + 1) * np + pt) * n;
            u64 *u0 = u + (size_t)t * n, *u1 = u + (size_t)(k + 1 + t) * n;
            for (int x = 0; x < n; x++) {
                u0[x] = addm(u0[x], mulm(dj[x], b[x], q), q);
                u1[x] = addm(u1[x], mulm(dj[x], a[x], q), q);
            }
        }
    }
    free(tmp);
}

/* Drop the last modulus of one polynomial given as [k+1][N] NTT form over moduli m_0..m_k
 * (m_k is P for ModDown, q_k for rescale): out_i = (x_i - lift(x_k)) * m_k^{-1} mod m_i,
 * i.e. round(x / m_k). */
static void drop_last(const or_ctx *c, int k, const int *primes, const u64 *x, u64 *out) {
    int n = c->n;
    int plast = primes[k];
    u64 ql = c->q[plast];
    u64 *coef = (u64 *)malloc(sizeof(u64) * n), *ext = (u64 *)malloc(sizeof(u64) * n);
    memcpy(coef, x + (size_t)k * n, sizeof(u64) * n);
    ntt_inv(c, plast, coef);
    for (int i = 0; i < k; i++) {
        int pi = primes[i];
        u64 q = c->q[pi], inv = invm(ql % q, q);
        for (int z = 0; z < n; z++) ext[z] = lift_centered(coef[z], ql, q);
        ntt_fwd(c, pi, ext);
        const u64 *xi = x + (size_t)i * n;
        u64 *o = out + (size_t)i * n;
        for (int z = 0; z < n; z++) o[z] = mulm(subm(xi[z], ext[z], q), inv, q);
    }
    free(coef); free(ext);
}

/* ModDown of a [2][k+1][N] extended pair into [2][k][N]. */
void or_moddown(const or_ctx *c, int k, const u64 *u, u64 *out) {
    int primes[OR_MAXP];
    for (int i = 0; i < k; i++) primes[i] = i;
    primes[k] = c->nq;
    for (int p = 0; p < 2; p++)
        drop_last(c, k, primes, u + (size_t)p * (k + 1) * c->n, out + (size_t)p * k * c->n);
}

/* Key switch of d ([k][N] NTT form) under key: returns (KS0, KS1) as [2][k][N]. */
void or_keyswitch(const or_ctx *c, int k, const u64 *d, const u64 *key, u64 *out) {
    int n = c->n;
    u64 *dig = (u64 *)malloc(sizeof(u64) * (size_t)k * (k + 1) * n);
    u64 *u = (u64 *)malloc(sizeof(u64) * 2 * (size_t)(k + 1) * n);
    or_modup(c, k, d, dig);
    key_inner(c, k, dig, key, 1, u);
    or_moddown(c, k, u, out);
    free(dig); free(u);
}

/* Rotation by Galois element g (unhoisted): (sigma(c0) + KS0(sigma(c1)), KS1(sigma(c1))). */
void or_rotate(const or_ctx *c, int k, const u64 *ct, const u64 *key, u64 g, u64 *out) {
    int n = c->n;
    size_t kn = (size_t)k * n;
    u64 *sc = (u64 *)malloc(sizeof(u64) * 2 * kn), *ks = (u64 *)malloc(sizeof(u64) * 2 * kn);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < k; i++)
            or_automorph_ntt(c, g, ct + p * kn + (size_t)i * n, sc + p * kn + (size_t)i * n);
    or_keyswitch(c, k, sc + kn, key, ks);
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        for (int x = 0; x < n; x++) {
            size_t o = (size_t)i * n + x;
            out[o] = addm(sc[o], ks[o], q);
            out[kn + o] = ks[kn + o];
        }
    }
    free(sc); free(ks);
}

/* Hoisted rotation: the ModUp digits of c1 are computed once by the caller; sigma_g is applied
 * to the digits and to c0. Bit-identical to or_rotate because the centered lift commutes with
 * the signed coefficient permutation. */
void or_rotate_hoisted(const or_ctx *c, int k, const u64 *ct, const u64 *digits, const u64 *key,
                       u64 g, u64 *out) {
    int n = c->n;
    size_t kn = (size_t)k * n;
    u64 *u = (u64 *)malloc(sizeof(u64) * 2 * (size_t)(k + 1) * n);
    u64 *ks = (u64 *)malloc(sizeof(u64) * 2 * kn), *t0 = (u64 *)malloc(sizeof(u64) * n);
    key_inner(c, k, digits, key, g, u);
    or_moddown(c, k, u, ks);
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        or_automorph_ntt(c, g, ct + (size_t)i * n, t0);
        for (int x = 0; x < n; x++) {
            size_t o = (size_t)i * n + x;
            out[o] = addm(t0[x], ks[o], q);
            out[kn + o] = ks[kn + o];
        }
    }
    free(u); free(ks); free(t0);
}

/* Rescale [2][k][N] -> [2][k-1][N]: divide by q_{k-1} with rounding. */
void or_rescale(const or_ctx *c, int k, const u64 *ct, u64 *out) {
    int primes[OR_MAXP];
    for (int i = 0; i < k; i++) primes[i] = i;
    for (int p = 0; p < 2; p++)
        drop_last(c, k - 1, primes, ct + (size_t)p * k * c->n, out + (size_t)p * (k - 1) * c->n);
}

/* ---------------------------------------------------------------- layer operations */

typedef struct {
    int count;
    const u64 *gs;          /* Galois elements */
    const u64 *const *keys; /* matching keys, [nq][2][np][N] each */
} keyset_t;

static const u64 *find_key(const keyset_t *ks, u64 g) {
    for (int i = 0; i < ks->count; i++) if (ks->gs[i] == g) return ks->keys[i];
    return NULL;
}

/* x^2 with relinearization and rescale: [2][k][N] -> [2][k-1][N]. */
int or_square(const or_ctx *c, int k, const u64 *ct, const u64 *rlk, u64 *out) {
    int n = c->n;
    size_t kn = (size_t)k * n;
    u64 *d = (u64 *)calloc(3 * kn, sizeof(u64)), *ks = (u64 *)calloc(2 * kn, sizeof(u64));
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        for (int x = 0; x < n; x++) {
            size_t o = (size_t)i * n + x;
            u64 a = ct[o], b = ct[kn + o];
            d[o] = mulm(a, a, q);
            d[kn + o] = mulm(addm(a, a, q), b, q);
            d[2 * kn + o] = mulm(b, b, q);
        }
    }
    or_keyswitch(c, k, d + 2 * kn, rlk, ks);
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        for (int x = 0; x < n; x++) {
            size_t o = (size_t)i * n + x;
            d[o] = addm(d[o], ks[o], q);
            d[kn + o] = addm(d[kn + o], ks[kn + o], q);
        }
    }
    or_rescale(c, k, d, out);
    free(d); free(ks);
    return 0;
}

/* The dense layer with its baby steps kept over Q*P ("double hoisting": Bossuat, Mouchet,
 * Troncoso-Pastoriza, Hubaux, Eurocrypt 2021). Every baby rotation stays in the extended basis,
 *   ct~_j = (key product of sigma_j(c1)) + (P sigma_j(c0), 0),   ct~_0 = P ct,
 * so that ModDown(ct~_j) = rot_j(ct) up to rounding; the plaintext products of Eq. (1) are taken
 * over Q*P with plaintexts that carry a residue mod P as well, and only then lowered:
 *   inner~_k2 = sum_j pt_{k2 t1 + j} ct~_j            (over Q*P)
 *   giant step k2 >= 1: its c1 is lowered (ModDown), rotated by sigma = 5^{k2 t1} and key
 *   switched; the key product plus sigma(c0 of inner~_k2) joins the extended sum,
 *   out = ModDown(inner~_0 + sum_{k2 >= 1} (KS_k2 + (sigma(c0~_k2), 0))), then the rescale.
 * The value is that of the other variants up to rounding (one ModDown per giant step plus one
 * at the end, instead of one per baby rotation). pts: [t][k+1][N] (row k mod P). */
static int dense_qp(const or_ctx *c, int k, const u64 *ct, const u64 *pts, int t1, int t2, int no_rescale,
                    const keyset_t *ks, u64 *out) {
    int n = c->n, nq = c->nq;
    size_t kn = (size_t)k * n, en = (size_t)(k + 1) * n, ecs = 2 * en;
    u64 *rots = (u64 *)calloc(ecs * t1, sizeof(u64));
    u64 *dig = (u64 *)malloc(sizeof(u64) * (size_t)k * (k + 1) * n);
    u64 *u = (u64 *)malloc(sizeof(u64) * ecs), *inner = (u64 *)malloc(sizeof(u64) * ecs);
    u64 *acc = (u64 *)calloc(ecs, sizeof(u64)), *low = (u64 *)malloc(sizeof(u64) * 2 * kn);
    u64 *i1 = (u64 *)malloc(sizeof(u64) * kn), *sc1 = (u64 *)malloc(sizeof(u64) * kn);
    u64 *tmp = (u64 *)malloc(sizeof(u64) * n);
    int primes[OR_MAXP], rc = 0;
    for (int i = 0; i < k; i++) primes[i] = i;
    primes[k] = nq;
    /* j = 0: P ct (zero mod P) */
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < k; i++) {
            u64 q = c->q[i], pm = c->q[nq] % q;
            for (int x = 0; x < n; x++) rots[p * en + (size_t)i * n + x] = mulm(pm, ct[p * kn + (size_t)i * n + x], q);
        }
    or_modup(c, k, ct + kn, dig);
    for (int j = 1; j < t1; j++) {
        u64 g = or_galois_elt(c, j);
        const u64 *key = find_key(ks, g);
        if (!key) { rc = -5; goto done; }
        key_inner(c, k, dig, key, g, u);
        u64 *r = rots + ecs * j;
        memcpy(r, u, sizeof(u64) * ecs);
        for (int i = 0; i < k; i++) {
            u64 q = c->q[i], pm = c->q[nq] % q;
            or_automorph_ntt(c, g, ct + (size_t)i * n, tmp);
            for (int x = 0; x < n; x++) r[(size_t)i * n + x] = addm(r[(size_t)i * n + x], mulm(pm, tmp[x], q), q);
        }
    }
    for (int k2 = 0; k2 < t2; k2++) {
        memset(inner, 0, sizeof(u64) * ecs);
        for (int j = 0; j < t1; j++) {
            const u64 *pt = pts + (size_t)(k2 * t1 + j) * en;
            const u64 *r = rots + ecs * j;
            for (int p = 0; p < 2; p++)
                for (int i = 0; i <= k; i++) {
                    u64 q = c->q[primes[i]];
                    for (int x = 0; x < n; x++) {
                        size_t o = (size_t)i * n + x;
                        inner[p * en + o] = addm(inner[p * en + o], mulm(pt[o], r[p * en + o], q), q);
                    }
                }
        }
        if (k2 == 0) {
            memcpy(acc, inner, sizeof(u64) * ecs);
            continue;
        }
        u64 g = or_galois_elt(c, (long)k2 * t1);
        const u64 *key = find_key(ks, g);
        if (!key) { rc = -5; goto done; }
        drop_last(c, k, primes, inner + en, i1);            /* c1 of the giant step, over Q */
        for (int i = 0; i < k; i++) or_automorph_ntt(c, g, i1 + (size_t)i * n, sc1 + (size_t)i * n);
        or_modup(c, k, sc1, dig);
        key_inner(c, k, dig, key, 1, u);
        for (int i = 0; i <= k; i++) {
            u64 q = c->q[primes[i]];
            or_automorph_ntt(c, g, inner + (size_t)i * n, tmp);
            for (int x = 0; x < n; x++) {
                size_t o = (size_t)i * n + x;
                acc[o] = addm(acc[o], addm(u[o], tmp[x], q), q);
                acc[en + o] = addm(acc[en + o], u[en + o], q);
            }
        }
    }
    or_moddown(c, k, acc, low);
    if (no_rescale) memcpy(out, low, sizeof(u64) * 2 * kn);
    else or_rescale(c, k, low, out);
done:
    free(rots); free(dig); free(u); free(inner); free(acc); free(low); free(i1); free(sc1); free(tmp);
    return rc;
}

/* Baby-step giant-step diagonal dense layer at k live primes (Eq. (1) of the paper):
 *   out = sum_{k2 < t2} rot_{k2 t1}( sum_{j < t1} pt_{k2 t1 + j} * rot_j(ct) ),
 * baby rotations hoisted, one rescale at the end. Giant steps: with lazy == 0 each rotation is a
 * full key switch with its own ModDown; with lazy != 0 the key inner products of all giant steps
 * are summed over Q*P and lowered by a single ModDown (same value up to rounding: one rounding of
 * the sum instead of one per giant step). pts: [t][k][N] NTT form. Returns -5 if a needed
 * rotation key is missing. flags: bit 0 = lazy giant steps; bit 1 = skip the final rescale and
 * return the [2][k][N] sum itself (used by tests to compare the variants); bit 2 = baby steps over
 * Q*P (dense_qp above; its giant steps are lowered by one final ModDown, and pts is [t][k+1][N]). */
int or_dense(const or_ctx *c, int k, const u64 *ct, const u64 *pts, int t, int t1, int flags,
             int n_keys, const u64 *gs, const u64 *const *keys, u64 *out) {
    const int lazy = flags & 1, no_rescale = flags & 2;
    int n = c->n, t2 = t / t1;
    size_t kn = (size_t)k * n, cts = 2 * kn;
    keyset_t ks = {n_keys, gs, keys};
    if (t1 * t2 != t) return -1;
    if (flags & 4) return dense_qp(c, k, ct, pts, t1, t2, no_rescale, &ks, out);
    u64 *rots = (u64 *)malloc(sizeof(u64) * cts * t1);
    u64 *dig = (u64 *)malloc(sizeof(u64) * (size_t)k * (k + 1) * n);
    u64 *inner = (u64 *)malloc(sizeof(u64) * cts), *acc = (u64 *)calloc(cts, sizeof(u64));
    u64 *tmp = (u64 *)malloc(sizeof(u64) * cts);
    size_t ext = 2 * (size_t)(k + 1) * n;
    u64 *usum = (u64 *)calloc(ext, sizeof(u64)), *u = (u64 *)malloc(sizeof(u64) * ext);
    u64 *sc1 = (u64 *)malloc(sizeof(u64) * kn);
    int rc = 0;
    memcpy(rots, ct, sizeof(u64) * cts);
    or_modup(c, k, ct + kn, dig);
    for (int j = 1; j < t1; j++) {
        u64 g = or_galois_elt(c, j);
        const u64 *key = find_key(&ks, g);
        if (!key) { rc = -5; goto done; }
        or_rotate_hoisted(c, k, ct, dig, key, g, rots + cts * j);
    }
    for (int k2 = 0; k2 < t2; k2++) {
        memset(inner, 0, sizeof(u64) * cts);
        for (int j = 0; j < t1; j++) {
            const u64 *pt = pts + (size_t)(k2 * t1 + j) * kn;
            const u64 *r = rots + cts * j;
            for (int p = 0; p < 2; p++)
                for (int i = 0; i < k; i++) {
                    u64 q = c->q[i];
                    for (int x = 0; x < n; x++) {
                        size_t o = (size_t)i * n + x;
                        inner[p * kn + o] = addm(inner[p * kn + o], mulm(pt[o], r[p * kn + o], q), q);
                    }
                }
        }
        const u64 *add = inner;
        if (k2 > 0 && lazy) {
            /* sigma_g(c0) joins the sum directly; sigma_g(c1) is raised and multiplied by the key,
             * and the product is accumulated over Q*P */
            u64 g = or_galois_elt(c, (long)k2 * t1);
            const u64 *key = find_key(&ks, g);
            if (!key) { rc = -5; goto done; }
            memset(tmp, 0, sizeof(u64) * cts);
            for (int i = 0; i < k; i++) {
                or_automorph_ntt(c, g, inner + (size_t)i * n, tmp + (size_t)i * n);
                or_automorph_ntt(c, g, inner + kn + (size_t)i * n, sc1 + (size_t)i * n);
            }
            or_modup(c, k, sc1, dig);
            key_inner(c, k, dig, key, 1, u);
            for (int p = 0; p < 2; p++)
                for (int i = 0; i <= k; i++) {
                    u64 q = c->q[ext_prime(k, i, c)];
                    for (int x = 0; x < n; x++) {
                        size_t o = ((size_t)p * (k + 1) + i) * n + x;
                        usum[o] = addm(usum[o], u[o], q);
                    }
                }
            add = tmp;
        } else if (k2 > 0) {
            u64 g = or_galois_elt(c, (long)k2 * t1);
            const u64 *key = find_key(&ks, g);
            if (!key) { rc = -5; goto done; }
            or_rotate(c, k, inner, key, g, tmp);
            add = tmp;
        }
        for (int p = 0; p < 2; p++)
            for (int i = 0; i < k; i++) {
                u64 q = c->q[i];
                for (int x = 0; x < n; x++) {
                    size_t o = p * kn + (size_t)i * n + x;
                    acc[o] = addm(acc[o], add[o], q);
                }
            }
    }
    if (lazy && t2 > 1) {
        or_moddown(c, k, usum, tmp);
        for (int p = 0; p < 2; p++)
            for (int i = 0; i < k; i++) {
                u64 q = c->q[i];
                for (int x = 0; x < n; x++) {
                    size_t o = p * kn + (size_t)i * n + x;
                    acc[o] = addm(acc[o], tmp[o], q);
                }
            }
    }
    if (no_rescale) memcpy(out, acc, sizeof(u64) * cts);
    else or_rescale(c, k, acc, out);
done:
    free(rots); free(dig); free(inner); free(acc); free(tmp); free(usum); free(u); free(sc1);
    return rc;
}

/* Replicate [y | 0] into [y | y]: ct + rot_{-w}(ct), same level. */
int or_replicate(const or_ctx *c, int k, const u64 *ct, int w, int n_keys, const u64 *gs,
                 const u64 *const *keys, u64 *out) {
    keyset_t ks = {n_keys, gs, keys};
    u64 g = or_galois_elt(c, -(long)w);
    const u64 *key = find_key(&ks, g);
    if (!key) return -5;
    size_t cts = 2 * (size_t)k * c->n;
    or_rotate(c, k, ct, key, g, out);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < k; i++) {
            u64 q = c->q[i];
            for (int x = 0; x < c->n; x++) {
                size_t o = (size_t)p * k * c->n + (size_t)i * c->n + x;
                out[o] = addm(out[o], ct[o], q);
            }
        }
    (void)cts;
    return 0;
}

/* Elementwise helpers exposed for tests. */
void or_mul_ntt(const or_ctx *c, int pi, const u64 *a, const u64 *b, u64 *out) {
    for (int x = 0; x < c->n; x++) out[x] = mulm(a[x], b[x], c->q[pi]);
}

void or_lift(const or_ctx *c, int from, int to, const u64 *in, u64 *out) {
    for (int x = 0; x < c->n; x++) out[x] = lift_centered(in[x], c->q[from], c->q[to]);
}

/* ---------------------------------------------------------------- layers of the paper's CNN */

/* Product of two ciphertexts at k primes (tensor, relinearization of the s^2 part, rescale):
 * [2][k][N] x [2][k][N] -> [2][k-1][N]. */
int or_mul(const or_ctx *c, int k, const u64 *a, const u64 *b, const u64 *rlk, u64 *out) {
    int n = c->n;
    size_t kn = (size_t)k * n;
    u64 *d = (u64 *)calloc(3 * kn, sizeof(u64)), *ks = (u64 *)calloc(2 * kn, sizeof(u64));
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        for (int x = 0; x < n; x++) {
            size_t o = (size_t)i * n + x;
            d[o] = mulm(a[o], b[o], q);
            d[kn + o] = addm(mulm(a[o], b[kn + o], q), mulm(a[kn + o], b[o], q), q);
            d[2 * kn + o] = mulm(a[kn + o], b[kn + o], q);
        }
    }
    or_keyswitch(c, k, d + 2 * kn, rlk, ks);
    for (int i = 0; i < k; i++) {
        u64 q = c->q[i];
        for (int x = 0; x < n; x++) {
            size_t o = (size_t)i * n + x;
            d[o] = addm(d[o], ks[o], q);
            d[kn + o] = addm(d[kn + o], ks[kn + o], q);
        }
    }
    or_rescale(c, k, d, out);
    free(d); free(ks);
    return 0;
}

/* A signed integer as a residue mod q. */
static u64 signed_mod(int64_t v, u64 q) {
    u64 m = (u64)(v < 0 ? -(v + 1) : v) % q;     /* |v| - 1 for negatives avoids INT64_MIN overflow */
    if (v < 0) m = negm(addm(m, 1 % q, q), q);
    return m;
}

/* ct * mul + add, where mul and add are signed integer constants: every residue is multiplied by
 * mul, and add (the constant polynomial, whose NTT form is add in every slot) is added to c0.
 * in: [2][k_in][N]; out: [2][k_out][N] with k_out <= k_in (the residues of primes >= k_out are
 * discarded, which keeps the value and lowers the level). */
void or_affine(const or_ctx *c, int k_in, int k_out, const u64 *in, int64_t mul, int64_t add, u64 *out) {
    int n = c->n;
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < k_out; i++) {
            u64 q = c->q[i], m = signed_mod(mul, q), a = p == 0 ? signed_mod(add, q) : 0;
            const u64 *src = in + ((size_t)p * k_in + i) * n;
            u64 *dst = out + ((size_t)p * k_out + i) * n;
            for (int x = 0; x < n; x++) dst[x] = addm(mulm(src[x], m, q), a, q);
        }
}

/* 1D convolution, packed single-channel (Section 3.1, "1D Convolutions"): with f taps and centre
 * h = (f - 1) / 2, out = rescale(sum_{i < f} pts_i * rot_{i - h}(ct)). One plaintext product per
 * tap and one rotation per tap but the centre one; the zero padding is carried by the plaintexts.
 * pts: [f][k][N] NTT form. */
int or_conv1d(const or_ctx *c, int k, const u64 *ct, const u64 *pts, int f, int n_keys, const u64 *gs,
              const u64 *const *keys, u64 *out) {
    keyset_t ks = {n_keys, gs, keys};
    int n = c->n, h = (f - 1) / 2;
    size_t kn = (size_t)k * n, cts = 2 * kn;
    u64 *acc = (u64 *)calloc(cts, sizeof(u64)), *r = (u64 *)malloc(sizeof(u64) * cts);
    int rc = 0;
    for (int i = 0; i < f; i++) {
        if (i == h) {
            memcpy(r, ct, sizeof(u64) * cts);
        } else {
            u64 g = or_galois_elt(c, (long)i - h);
            const u64 *key = find_key(&ks, g);
            if (!key) { rc = -5; goto done; }
            or_rotate(c, k, ct, key, g, r);
        }
        const u64 *pt = pts + (size_t)i * kn;
        for (int p = 0; p < 2; p++)
            for (int j = 0; j < k; j++) {
                u64 q = c->q[j];
                for (int x = 0; x < n; x++) {
                    size_t o = (size_t)j * n + x;
                    acc[p * kn + o] = addm(acc[p * kn + o], mulm(pt[o], r[p * kn + o], q), q);
                }
            }
    }
    or_rescale(c, k, acc, out);
done:
    free(acc); free(r);
    return rc;
}

/* Average pool, stride 1, size f (Section 3.1, "Average Pool"): s = sum_{i < f} rot_{-i}(ct)
 * (f - 1 rotations), then one plaintext product with pt (1/f on the valid outputs, 0 elsewhere)
 * and a rescale. pt: [k][N] NTT form. */
/* sum_j pts_j * ct~_{rots_j} over Q*P ([2][k+1][N] into acc): ct~_0 = P ct for rotation 0, else the
 * hoisted key product of sigma(c1) plus (P sigma(c0), 0) (the baby steps of dense_qp).
 * pts: [n][k+1][N] (row k mod P), or a single plaintext for every term when pt_stride is 0. */
static int qp_rotation_sum(const or_ctx *c, int k, const u64 *ct, const long *rots, int n_rot, const u64 *pts,
                           size_t pt_stride, const keyset_t *ks, u64 *acc) {
    int n = c->n, nq = c->nq;
    size_t kn = (size_t)k * n, en = (size_t)(k + 1) * n, ecs = 2 * en;
    u64 *dig = (u64 *)malloc(sizeof(u64) * (size_t)k * (k + 1) * n);
    u64 *r = (u64 *)malloc(sizeof(u64) * ecs), *tmp = (u64 *)malloc(sizeof(u64) * n);
    int primes[OR_MAXP], rc = 0;
    for (int i = 0; i < k; i++) primes[i] = i;
    primes[k] = nq;
    memset(acc, 0, sizeof(u64) * ecs);
    or_modup(c, k, ct + kn, dig);
    for (int j = 0; j < n_rot; j++) {
        if (rots[j] == 0) {
            memset(r, 0, sizeof(u64) * ecs);
            for (int p = 0; p < 2; p++)
                for (int i = 0; i < k; i++) {
                    u64 q = c->q[i], pm = c->q[nq] % q;
                    for (int x = 0; x < n; x++) r[p * en + (size_t)i * n + x] = mulm(pm, ct[p * kn + (size_t)i * n + x], q);
                }
        } else {
            u64 g = or_galois_elt(c, rots[j]);
            const u64 *key = find_key(ks, g);
            if (!key) { rc = -5; goto done; }
            key_inner(c, k, dig, key, g, r);
            for (int i = 0; i < k; i++) {
                u64 q = c->q[i], pm = c->q[nq] % q;
                or_automorph_ntt(c, g, ct + (size_t)i * n, tmp);
                for (int x = 0; x < n; x++) r[(size_t)i * n + x] = addm(r[(size_t)i * n + x], mulm(pm, tmp[x], q), q);
            }
        }
        const u64 *pt = pts + pt_stride * j;
        for (int p = 0; p < 2; p++)
            for (int i = 0; i <= k; i++) {
                u64 q = c->q[primes[i]];
                for (int x = 0; x < n; x++) {
                    size_t o = (size_t)i * n + x;
                    acc[p * en + o] = addm(acc[p * en + o], mulm(pt[o], r[p * en + o], q), q);
                }
            }
    }
done:
    free(dig); free(r); free(tmp);
    return rc;
}

/* Convolution with its rotations kept over Q*P (the baby steps of dense_qp, one ModDown of the
 * sum): ModDown(sum_i pts_i * ct~_{i-(f-1)/2}), then the rescale. pts: [f][k+1][N]. */
int or_conv1d_qp(const or_ctx *c, int k, const u64 *ct, const u64 *pts, int f, int n_keys, const u64 *gs,
                 const u64 *const *keys, u64 *out) {
    keyset_t ks = {n_keys, gs, keys};
    int n = c->n, h = (f - 1) / 2;
    size_t en = (size_t)(k + 1) * n;
    long rots[64];
    if (f > 64) return -1;
    for (int i = 0; i < f; i++) rots[i] = (long)i - h;
    u64 *acc = (u64 *)malloc(sizeof(u64) * 2 * en), *low = (u64 *)malloc(sizeof(u64) * 2 * (size_t)k * n);
    int rc = qp_rotation_sum(c, k, ct, rots, f, pts, en, &ks, acc);
    if (!rc) {
        or_moddown(c, k, acc, low);
        or_rescale(c, k, low, out);
    }
    free(acc); free(low);
    return rc;
}

/* Average pool with its rotations kept over Q*P: ModDown(pt * sum_{i<f} ct~_{-i}) (the products
 * summed term by term, the same residues by distributivity), then the rescale. pt: [k+1][N]. */
int or_avgpool_qp(const or_ctx *c, int k, const u64 *ct, const u64 *pt, int f, int n_keys, const u64 *gs,
                  const u64 *const *keys, u64 *out) {
    keyset_t ks = {n_keys, gs, keys};
    int n = c->n;
    size_t en = (size_t)(k + 1) * n;
    long rots[64];
    if (f > 64) return -1;
    for (int i = 0; i < f; i++) rots[i] = -(long)i;
    u64 *acc = (u64 *)malloc(sizeof(u64) * 2 * en), *low = (u64 *)malloc(sizeof(u64) * 2 * (size_t)k * n);
    int rc = qp_rotation_sum(c, k, ct, rots, f, pt, 0, &ks, acc);
    if (!rc) {
        or_moddown(c, k, acc, low);
        or_rescale(c, k, low, out);
    }
    free(acc); free(low);
    return rc;
}

int or_avgpool(const or_ctx *c, int k, const u64 *ct, const u64 *pt, int f, int n_keys, const u64 *gs,
               const u64 *const *keys, u64 *out) {
    keyset_t ks = {n_keys, gs, keys};
    int n = c->n;
    size_t kn = (size_t)k * n, cts = 2 * kn;
    u64 *s = (u64 *)malloc(sizeof(u64) * cts), *r = (u64 *)malloc(sizeof(u64) * cts);
    int rc = 0;
    memcpy(s, ct, sizeof(u64) * cts);
    for (int i = 1; i < f; i++) {
        u64 g = or_galois_elt(c, -(long)i);
        const u64 *key = find_key(&ks, g);
        if (!key) { rc = -5; goto done; }
        or_rotate(c, k, ct, key, g, r);
        for (int p = 0; p < 2; p++)
            for (int j = 0; j < k; j++) {
                u64 q = c->q[j];
                for (int x = 0; x < n; x++) {
                    size_t o = p * kn + (size_t)j * n + x;
                    s[o] = addm(s[o], r[o], q);
                }
            }
    }
    for (int p = 0; p < 2; p++)
        for (int j = 0; j < k; j++) {
            u64 q = c->q[j];
            for (int x = 0; x < n; x++) {
                size_t o = (size_t)j * n + x;
                s[p * kn + o] = mulm(s[p * kn + o], pt[o], q);
            }
        }
    or_rescale(c, k, s, out);
done:
    free(s); free(r);
    return rc;
}

/* Integer constants of the degree-3 activation c0 + c1 z + c2 z^2 + c3 z^3 on z at k primes and
 * scale S (q_a = q_{k-1}, q_b = q_{k-2} are the primes its two rescales drop):
 *   S2 = S S / q_a                      scale of z^2 and of (c3 z + c2)
 *   S3 = S2 S2 / q_b                    output scale
 *   C3 = llround(c3 S), C2 = llround(c2 S2), C1 = llround(c1 (S3 q_a / S)), C0 = llround(c0 S3).
 * Returns S3. */
double or_poly3_consts(const or_ctx *c, int k, double S, const double *coef, int64_t *C) {
    double qa = (double)c->q[k - 1], qb = (double)c->q[k - 2];
    double S2 = (S * S) / qa;
    double S3 = (S2 * S2) / qb;
    C[3] = llround(coef[3] * S);
    C[2] = llround(coef[2] * S2);
    C[1] = llround(coef[1] * ((S3 * qa) / S));
    C[0] = llround(coef[0] * S3);
    return S3;
}

/* Degree-3 polynomial activation with depth 2 (the ReLU approximation of Section 3.1):
 *   z2 = rescale(relin(z z))                        k-1 primes, scale S2
 *   u  = rescale(z C3) + C2                         k-1 primes, scale S2  (c3 z + c2)
 *   w  = rescale(relin(z2 u))                       k-2 primes, scale S3  (c3 z^3 + c2 z^2)
 *   v  = drop(rescale(z C1)) + C0                   k-2 primes, scale S3  (c1 z + c0)
 *   out = w + v.
 * ct: [2][k][N] (k >= 3); out: [2][k-2][N]. Returns the output scale. */
double or_poly3(const or_ctx *c, int k, const u64 *ct, double S, const double *coef, const u64 *rlk, u64 *out) {
    int n = c->n;
    size_t kn = (size_t)k * n, k1 = (size_t)(k - 1) * n, k2 = (size_t)(k - 2) * n;
    int64_t C[4];
    double S3 = or_poly3_consts(c, k, S, coef, C);
    u64 *z2 = (u64 *)malloc(sizeof(u64) * 2 * k1), *t = (u64 *)malloc(sizeof(u64) * 2 * kn);
    u64 *u = (u64 *)malloc(sizeof(u64) * 2 * k1), *w = (u64 *)malloc(sizeof(u64) * 2 * k2);
    or_square(c, k, ct, rlk, z2);
    or_affine(c, k, k, ct, C[3], 0, t);
    or_rescale(c, k, t, u);
    or_affine(c, k - 1, k - 1, u, 1, C[2], u);
    or_mul(c, k - 1, z2, u, rlk, w);
    or_affine(c, k, k, ct, C[1], 0, t);
    or_rescale(c, k, t, u);
    or_affine(c, k - 1, k - 2, u, 1, C[0], out);
    for (int p = 0; p < 2; p++)
        for (int i = 0; i < k - 2; i++) {
            u64 q = c->q[i];
            for (int x = 0; x < n; x++) {
                size_t o = p * k2 + (size_t)i * n + x;
                out[o] = addm(out[o], w[o], q);
            }
        }
    free(z2); free(t); free(u); free(w);
    return S3;
}

/* ---------------------------------------------------------------- seeded symmetric encryption */

/* Secret-key encryption at the top level: ct = (-a s + e + m, a), [2][nq][N] NTT form, with a
 * uniform drawn directly as NTT values prime by prime from the stream (seed, TAG_SYM_A, 0) and e
 * Gaussian from (seed, TAG_SYM_E, 0). c1 = a is a function of the seed alone, so the client can
 * send c0 and the seed (half the bytes) and the server regenerates c1. */
void or_encrypt_sym(const or_ctx *c, const int64_t *s, const int64_t *m, u64 seed, u64 *ct) {
    int n = c->n, nq = c->nq;
    int64_t *e = (int64_t *)malloc(sizeof(int64_t) * n);
    u64 *sn = (u64 *)malloc(sizeof(u64) * n), *tn = (u64 *)malloc(sizeof(u64) * n);
    stream_t sa, se;
    stream_init(&sa, seed, TAG_SYM_A, 0);
    stream_init(&se, seed, TAG_SYM_E, 0);
    sample_gauss(c, &se, n, e);
    for (int i = 0; i < nq; i++) {
        u64 q = c->q[i];
        u64 *c0 = ct + (size_t)i * n, *a = ct + (size_t)(nq + i) * n;
        for (int k = 0; k < n; k++) a[k] = sample_uniform1(&sa, q);
        small_to_ntt(c, i, s, sn);
        small_to_ntt(c, i, e, c0);
        small_to_ntt(c, i, m, tn);
        for (int k = 0; k < n; k++) c0[k] = addm(subm(c0[k], mulm(a[k], sn[k], q), q), tn[k], q);
    }
    free(e); free(sn); free(tn);
}
