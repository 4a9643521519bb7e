// Host-side parameter derivation, ChaCha20 sampling, FP64 encoder and CRT for libcryptotl.
//
// Readings (the paper fixes none of these; CKKS is used as a black box in Section 3.1):
//   primes   for each bit size b in listed order, then the special prime: the largest prime
//            q < 2^b with q = 1 (mod 2N) not already taken
//   psi      the smallest primitive 2N-th root of unity mod q
//   sampler  ChaCha20 keyed by the 64-bit seed (little-endian, zero-padded to 32 bytes), nonce
//            (purpose tag, index low, index high), block counter from 0; ternary by bytes with
//            255 rejected and value (b mod 3) - 1; Gaussian by a 53-bit cumulative table over
//            -19..19; uniform mod q by 64-bit words with rejection at or above floor(2^64/q) q
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "ctl_internal.h"

namespace ctl {

u64 h_mulmod(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 h_powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q, x = a % q;
    for (; e; e >>= 1) {
        if (e & 1) r = h_mulmod(r, x, q);
        x = h_mulmod(x, x, q);
    }
    return r;
}

u64 h_invmod(u64 a, u64 q) { return h_powmod(a, q - 2, q); }

u64 h_shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

// Miller-Rabin with bases {2, 325, 9375, 28178, 450775, 9780504, 1795265022}: exact below 2^64.
static bool prime_u64(u64 n) {
    if (n < 2) return false;
    static const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : small) {
        if (n % p == 0) return n == p;
    }
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; ++s; }
    static const u64 bases[] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
    for (u64 a : bases) {
        a %= n;
        if (!a) continue;
        u64 x = h_powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < s && comp; ++i) {
            x = h_mulmod(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

static u64 smallest_psi(u64 q, int logn) {
    const u64 n = 1ull << logn, m = 2 * n;
    u64 root = 0;
    for (u64 x = 2; x < q; ++x) {
        root = h_powmod(x, (q - 1) / m, q);
        if (h_powmod(root, n, q) == q - 1) break;
    }
    // every primitive 2N-th root is an odd power of `root`
    const u64 r2 = h_mulmod(root, root, q);
    u64 best = root, cur = root;
    for (u64 e = 1; e < m; e += 2) {
        best = cur < best ? cur : best;
        cur = h_mulmod(cur, r2, q);
    }
    return best;
}

int derive_params(const ctl_params *p, HostParams *out, std::string *err) {
    if (!p) { *err = "null params"; return CTL_EINVAL; }
    if (p->log2n < 12 || p->log2n > 14) { *err = "log2n must be 12, 13 or 14"; return CTL_EPARAM; }
    if (p->n_q < 1 || p->n_q > CTL_MAX_PRIMES) { *err = "n_q out of range"; return CTL_EPARAM; }
    if (!(p->sigma > 0.0) || p->sigma > 100.0) { *err = "sigma out of range"; return CTL_EPARAM; }
    HostParams h;
    h.logn = p->log2n;
    h.n = 1 << h.logn;
    h.nq = p->n_q;
    h.np = p->n_q + 1;
    h.sigma = p->sigma;
    h.log2_scale = p->log2_scale;
    const u64 m = 2ull * h.n;
    for (int i = 0; i < h.np; ++i) {
        int b = i < h.nq ? p->q_bits[i] : p->p_bits;
        if (b < h.logn + 2 || b > 61) { *err = "prime bit size out of range"; return CTL_EPARAM; }
        u64 c = (1ull << b) - m + 1;
        for (;;) {
            bool taken = false;
            for (u64 t : h.mods) taken |= (t == c);
            if (!taken && prime_u64(c)) break;
            if (c <= m + 1) { *err = "no prime found"; return CTL_EPARAM; }
            c -= m;
        }
        h.mods.push_back(c);
    }
    for (int i = 0; i < h.np; ++i) h.psi.push_back(smallest_psi(h.mods[i], h.logn));
    // discrete Gaussian cumulative table: weights exp(-e^2 / (2 sigma^2)) for e = -19..19,
    // running sums in increasing e divided by the total, scaled by 2^53 and truncated
    double w[kCdtSize], total = 0.0, run = 0.0;
    for (int i = 0; i < kCdtSize; ++i) {
        double e = (double)(i - kGaussTail);
        w[i] = std::exp(-(e * e) / (2.0 * h.sigma * h.sigma));
    }
    for (int i = 0; i < kCdtSize; ++i) total += w[i];
    for (int i = 0; i < kCdtSize; ++i) {
        run += w[i];
        h.cdt[i] = (u64)std::ldexp(run / total, 53);
    }
    h.cdt[kCdtSize - 1] = 1ull << 53;
    *out = h;
    return CTL_OK;
}

u64 galois_elt(int logn, long r) {
    const long half = 1L << (logn - 1);
    long e = ((r % half) + half) % half;
    const u64 m = 2ull << logn;
    u64 g = 1, base = 5;
    for (; e; e >>= 1) {              // square-and-multiply of 5 modulo 2N
        if (e & 1) g = g * base % m;
        base = base * base % m;
    }
    return g;
}

u64 galois_inv(int logn, u64 g) {
    const u64 m = 2ull << logn;       // the odd residues mod 2N form a group of order N
    u64 r = 1, base = g % m;
    for (u64 e = (1ull << logn) - 1; e; e >>= 1) {
        if (e & 1) r = r * base % m;
        base = base * base % m;
    }
    return r;
}

// ---------------------------------------------------------------- ChaCha20
static inline uint32_t rotl(uint32_t v, int s) { return (v << s) | (v >> (32 - s)); }

static inline void quarter(uint32_t *x, int a, int b, int c, int d) {
    x[a] += x[b]; x[d] = rotl(x[d] ^ x[a], 16);
    x[c] += x[d]; x[b] = rotl(x[b] ^ x[c], 12);
    x[a] += x[b]; x[d] = rotl(x[d] ^ x[a], 8);
    x[c] += x[d]; x[b] = rotl(x[b] ^ x[c], 7);
}

void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint8_t out[64]) {
    uint32_t init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                         key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                         counter, nonce[0], nonce[1], nonce[2]};
    uint32_t x[16];
    std::memcpy(x, init, sizeof(x));
    for (int round = 0; round < 10; ++round) {
        quarter(x, 0, 4, 8, 12); quarter(x, 1, 5, 9, 13);
        quarter(x, 2, 6, 10, 14); quarter(x, 3, 7, 11, 15);
        quarter(x, 0, 5, 10, 15); quarter(x, 1, 6, 11, 12);
        quarter(x, 2, 7, 8, 13); quarter(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; ++i) {
        uint32_t v = x[i] + init[i];
        out[4 * i] = (uint8_t)v;
        out[4 * i + 1] = (uint8_t)(v >> 8);
        out[4 * i + 2] = (uint8_t)(v >> 16);
        out[4 * i + 3] = (uint8_t)(v >> 24);
    }
}

Stream::Stream(u64 seed, uint32_t tag, u64 index) : counter_(0), pos_(64) {
    std::memset(key_, 0, sizeof(key_));
    key_[0] = (uint32_t)seed;
    key_[1] = (uint32_t)(seed >> 32);
    nonce_[0] = tag;
    nonce_[1] = (uint32_t)index;
    nonce_[2] = (uint32_t)(index >> 32);
}

void Stream::refill() {
    chacha20_block(key_, counter_++, nonce_, buf_);
    pos_ = 0;
}

uint8_t Stream::byte() {
    if (pos_ == 64) refill();
    return buf_[pos_++];
}

u64 Stream::word() {
    u64 v = 0;
    for (int i = 0; i < 8; ++i) v |= (u64)byte() << (8 * i);
    return v;
}

void Stream::ternary(int n, int64_t *out) {
    for (int i = 0; i < n; ++i) {
        uint8_t b = byte();
        while (b == 255) b = byte();
        out[i] = (int64_t)(b % 3) - 1;
    }
}

void Stream::gaussian(const u64 *cdt, int n, int64_t *out) {
    for (int i = 0; i < n; ++i) {
        const u64 u = word() >> 11;
        int lo = 0;
        while (u >= cdt[lo]) ++lo;     // cdt[last] = 2^53 > u always stops the scan
        out[i] = (int64_t)lo - kGaussTail;
    }
}

u64 Stream::uniform(u64 q) {
    const u64 lim = (u64)(((u128)1 << 64) / q) * q;
    u64 x = word();
    while (x >= lim) x = word();
    return x % q;
}

// ---------------------------------------------------------------- encoder
Encoder::Encoder(int logn) : logn_(logn), n_(1 << logn) {
    const int m = 2 * n_;
    slot_exp_.resize(n_ / 2);
    int e = 1;
    for (int j = 0; j < n_ / 2; ++j) {
        slot_exp_[j] = e;
        e = (int)((long)e * 5 % m);
    }
    cs_.resize(m);
    sn_.resize(m);
    for (int k = 0; k < m; ++k) {
        cs_[k] = std::cos(M_PI * k / n_);
        sn_[k] = std::sin(M_PI * k / n_);
    }
}

// In-place iterative radix-2 DFT of length 2N: X[e] = sum_k x[k] exp(-+ i pi e k / N).
void Encoder::fft(std::vector<double> &re, std::vector<double> &im, bool inverse) const {
    const int m = 2 * n_, bits = logn_ + 1;
    for (int i = 0; i < m; ++i) {
        int r = 0;
        for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
        if (r > i) { std::swap(re[i], re[r]); std::swap(im[i], im[r]); }
    }
    const double sgn = inverse ? 1.0 : -1.0;
    for (int len = 2; len <= m; len <<= 1) {
        const int step = m / len;     // exp(-+ 2 pi i k / len) = exp(-+ i pi (k step) / N)
        for (int s = 0; s < m; s += len) {
            for (int k = 0; k < len / 2; ++k) {
                const int t = k * step;                    // < N
                const double c = cs_[t], si = sgn * sn_[t];
                const int a = s + k, b = s + k + len / 2;
                const double xr = re[b] * c - im[b] * si;
                const double xi = re[b] * si + im[b] * c;
                re[b] = re[a] - xr;
                im[b] = im[a] - xi;
                re[a] += xr;
                im[a] += xi;
            }
        }
    }
}

// m_k = (1/N) sum over odd e of w_e zeta^{-e k}, with w_{5^j} = z_j and w_{-5^j} = z_j (real z).
void Encoder::encode_real(const double *z, double *m) const {
    const int two_n = 2 * n_;
    std::vector<double> re(two_n, 0.0), im(two_n, 0.0);
    for (int j = 0; j < n_ / 2; ++j) {
        re[slot_exp_[j]] = z[j];
        re[two_n - slot_exp_[j]] = z[j];
    }
    fft(re, im, false);
    for (int k = 0; k < n_; ++k) m[k] = re[k] / n_;
}

// z_j = sum_k m_k zeta^{5^j k}: a length-2N DFT with positive exponent of m padded with zeros.
void Encoder::decode_real(const double *m, double *z) const {
    const int two_n = 2 * n_;
    std::vector<double> re(two_n, 0.0), im(two_n, 0.0);
    for (int k = 0; k < n_; ++k) re[k] = m[k];
    fft(re, im, true);
    for (int j = 0; j < n_ / 2; ++j) z[j] = re[slot_exp_[j]];
}

// ---------------------------------------------------------------- CRT
// Little-endian multi-limb unsigned integers, enough for 17 primes of 61 bits.
namespace {
struct Big {
    u64 w[18];
    int len;
};

void big_set(Big &a, u64 v) { a.w[0] = v; a.len = 1; }

void big_mul_add(Big &a, u64 m, u64 add) {     // a = a * m + add
    u128 carry = add;
    for (int i = 0; i < a.len; ++i) {
        u128 t = (u128)a.w[i] * m + carry;
        a.w[i] = (u64)t;
        carry = t >> 64;
    }
    if (carry) a.w[a.len++] = (u64)carry;
}

int big_cmp(const Big &a, const Big &b) {
    int la = a.len, lb = b.len;
    while (la > 1 && !a.w[la - 1]) --la;
    while (lb > 1 && !b.w[lb - 1]) --lb;
    if (la != lb) return la < lb ? -1 : 1;
    for (int i = la - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

void big_sub(Big &a, const Big &b) {          // a -= b, a >= b
    u64 borrow = 0;
    for (int i = 0; i < a.len; ++i) {
        u64 bi = i < b.len ? b.w[i] : 0;
        u128 t = (u128)a.w[i] - bi - borrow;
        a.w[i] = (u64)t;
        borrow = (u64)(t >> 64) ? 1 : 0;
    }
}

double big_to_double(const Big &a) {
    double v = 0.0;
    for (int i = a.len - 1; i >= 0; --i) v = v * 18446744073709551616.0 + (double)a.w[i];
    return v;
}
}  // namespace

double crt_centered_double(const u64 *r, const u64 *mods, int k) {
    // Garner: x = v_0 + q_0 (v_1 + q_1 (v_2 + ...)), v_i in [0, q_i)
    u64 v[kMaxMods];
    for (int i = 0; i < k; ++i) {
        u64 t = r[i] % mods[i];
        for (int j = 0; j < i; ++j) {
            u64 d = t >= v[j] % mods[i] ? t - v[j] % mods[i] : t + mods[i] - v[j] % mods[i];
            t = h_mulmod(d, h_invmod(mods[j] % mods[i], mods[i]), mods[i]);
        }
        v[i] = t;
    }
    Big x, q, half;
    big_set(x, v[k - 1]);
    for (int i = k - 2; i >= 0; --i) big_mul_add(x, mods[i], v[i]);
    big_set(q, 1);
    for (int i = 0; i < k; ++i) big_mul_add(q, mods[i], 0);
    // x > (Q - 1) / 2  <=>  2x > Q - 1  <=>  2x >= Q (Q odd)
    Big x2 = x;
    big_mul_add(x2, 2, 0);
    if (big_cmp(x2, q) >= 0) {
        Big d = q;
        d.len = q.len;
        big_sub(d, x);
        return -big_to_double(d);
    }
    (void)half;
    return big_to_double(x);
}

}  // namespace ctl
