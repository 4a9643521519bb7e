// Internal declarations shared by the host code and the HIP kernels of libcryptotl.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/ctl.h"

namespace ctl {

typedef unsigned long long u64;
typedef unsigned __int128 u128;

constexpr int kMaxMods = CTL_MAX_PRIMES + 1;   // ciphertext primes + special prime
constexpr int kGaussTail = 19;
constexpr int kCdtSize = 2 * kGaussTail + 1;

// ---------------------------------------------------------------- device-side constant tables
struct PrimeConst {
    u64 q;
    u64 q2;        // 2q
    u64 r64;       // 2^64 mod q
    u64 r64s;      // Shoup companion of r64
    u64 ones;      // floor(2^64 / q): Shoup companion of 1
    u64 ninv;      // N^{-1} mod q
    u64 ninvs;
    u64 qn;        // 2^64 - q
    u64 nq2;       // 2^64 - 2q
    u64 r60;       // 2^60 mod q for q below 2^60 (2^60 otherwise)
    u64 r60s;      // Shoup companion of r60 (q below 2^60)
    // FP64 arithmetic for primes below 2^41 (exact: see the kernels): fp != 0 selects it, and the
    // Shoup-companion twiddle tables of such a prime hold the twiddles as doubles instead.
    int fp;
    int pad_;
    double qd;     // q as a double
    double qinv;   // fl(1 / q)
    double ninvd;  // N^{-1} mod q as a double
};

constexpr u64 kFpPrimeLimit = 1ull << 41;

struct CrossConst {        // entry [i][j]: moving a value from modulus j to modulus i
    u64 qj_mod_qi;
    u64 inv;               // q_j^{-1} mod q_i
    u64 invs;
    double invd;           // inv as a double
};

// ---------------------------------------------------------------- host parameter math
struct HostParams {
    int logn = 0, n = 0, nq = 0, np = 0;
    std::vector<u64> mods;        // q_0..q_{nq-1}, P
    std::vector<u64> psi;
    double sigma = 3.2;
    int log2_scale = 0;
    u64 cdt[kCdtSize];
};

int derive_params(const ctl_params *p, HostParams *out, std::string *err);
u64 h_mulmod(u64 a, u64 b, u64 q);
u64 h_powmod(u64 a, u64 e, u64 q);
u64 h_invmod(u64 a, u64 q);
u64 h_shoup(u64 w, u64 q);
u64 galois_elt(int logn, long r);
u64 galois_inv(int logn, u64 g);    // g^{-1} mod 2N

// ChaCha20 stream (RFC 8439 block function) with the sampler conventions.
enum : uint32_t { TAG_SK = 1, TAG_PK_A = 2, TAG_PK_E = 3, TAG_KS_A = 4, TAG_KS_E = 5,
                  TAG_ENC_V = 8, TAG_ENC_E0 = 9, TAG_ENC_E1 = 10, TAG_SYM_A = 11, TAG_SYM_E = 12 };

class Stream {
  public:
    Stream(u64 seed, uint32_t tag, u64 index);
    uint8_t byte();
    u64 word();
    void ternary(int n, int64_t *out);
    void gaussian(const u64 *cdt, int n, int64_t *out);
    u64 uniform(u64 q);
  private:
    void refill();
    uint32_t key_[8], nonce_[3], counter_;
    uint8_t buf_[64];
    int pos_;
};
void chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint8_t out[64]);

// FP64 canonical-embedding encoder.
class Encoder {
  public:
    explicit Encoder(int logn);
    // unrounded coefficients m_k of the real slot vector z (N/2 entries)
    void encode_real(const double *z, double *m) const;
    // slots z_j from real coefficients m (N entries), real part
    void decode_real(const double *m, double *z) const;
  private:
    void fft(std::vector<double> &re, std::vector<double> &im, bool inverse) const;
    int logn_, n_;
    std::vector<int> slot_exp_;     // 5^j mod 2N
    std::vector<double> cs_, sn_;   // cos/sin(pi k / N), k < 2N
};

// Centered CRT of residues r[i] (i < k) modulo mods[0..k-1], returned as a double.
double crt_centered_double(const u64 *r, const u64 *mods, int k);

}  // namespace ctl
