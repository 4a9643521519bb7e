// HIP kernels of libcryptotl for CDNA4 (gfx950, wave64).
//
// All arithmetic is exact modular integer arithmetic on 64-bit residues (primes < 2^61), done on
// the integer VALU: products by fixed operands (twiddles, inverses) use Shoup's precomputed
// quotient, products of two variables and sums of products use a 128-bit accumulator reduced
// once (2^64 mod q and floor(2^64/q) as Shoup constants). No matrix cores: nothing here is a
// floating-point contraction.
//
// NTT layout: negacyclic, bit-reversed evaluation order (slot i = a(psi^{2 brv(i)+1})), computed
// with Cooley-Tukey butterflies forward and Gentleman-Sande inverse, twiddles psi^{brv(m)} taken
// from per-prime tables. One workgroup transforms one residue polynomial: N/16 threads hold 16
// values each in registers; each pass runs 4 (or 3) butterfly stages in registers and exchanges
// through LDS between passes, so a residue makes a single HBM round trip.
#include <map>
#include <mutex>
#include <type_traits>

#include "ctl_internal.h"
#include "kernels.h"

namespace ctl {

// ---------------------------------------------------------------- device arithmetic
// 64-bit residues on the 32-bit integer VALU. Products are assembled from v_mad_u64_u32
// (32 x 32 + 64 -> 64) so that carries stay inside the multiply-add instead of VCC carry chains.
typedef unsigned int u32;

__device__ __forceinline__ u64 mad32(u32 a, u32 b, u64 c) { return (u64)a * b + c; }

// high 64 bits of x * y
__device__ __forceinline__ u64 mulhi(u64 x, u64 y) {
    const u32 x0 = (u32)x, x1 = (u32)(x >> 32), y0 = (u32)y, y1 = (u32)(y >> 32);
    const u64 t = mad32(x0, y1, __umulhi(x0, y0));
    const u64 u = mad32(x1, y0, (u32)t);
    return mad32(x1, y1, t >> 32) + (u >> 32);
}

// x * w mod q, result in [0, 2q), for any x < 2^64 and w < q with ws = floor(w 2^64 / q):
// r = x w - floor(x ws / 2^64) q, computed mod 2^64 as x w + h (2^64 - q) (qn = 2^64 - q).
__device__ __forceinline__ u64 shoup_lazy(u64 x, u64 w, u64 ws, u64 q, u64 qn) {
    const u64 h = mulhi(x, ws);
    const u32 x0 = (u32)x, x1 = (u32)(x >> 32), w0 = (u32)w, w1 = (u32)(w >> 32);
    const u32 h0 = (u32)h, h1 = (u32)(h >> 32), n0 = (u32)qn, n1 = (u32)(qn >> 32);
    const u64 lo = mad32(h0, n0, (u64)x0 * w0);
    const u32 cross = x0 * w1 + x1 * w0 + h0 * n1 + h1 * n0;
    (void)q;
    return lo + ((u64)cross << 32);
}

// x - m if x >= m else x, for x, m < 2^63, from the sign of x - m (nm = 2^64 - m): one 64-bit
// add, one compare of the high word and two selects.
__device__ __forceinline__ u64 csub(u64 x, u64 nm) {
    const u64 d = x + nm;
    return (int)(u32)(d >> 32) < 0 ? x : d;
}

__device__ __forceinline__ u64 red2(u64 x, u64 q) { return x >= q ? x - q : x; }
__device__ __forceinline__ u64 red4(u64 x, u64 q, u64 q2) {
    x = x >= q2 ? x - q2 : x;
    return x >= q ? x - q : x;
}
__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) { return red2(a + b, q); }
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
__device__ __forceinline__ u64 neg_mod(u64 a, u64 q) { return a ? q - a : 0; }

struct Acc {
    u64 lo, hi;
};
__device__ __forceinline__ void acc_zero(Acc &a) { a.lo = 0; a.hi = 0; }
__device__ __forceinline__ void acc_mac(Acc &a, u64 x, u64 y) {
    const u64 l = x * y, h = mulhi(x, y);
    a.lo += l;
    a.hi += h + (a.lo < l ? 1ull : 0ull);
}
// (hi 2^64 + lo) mod q
__device__ __forceinline__ u64 acc_reduce(const Acc &a, const PrimeConst &p) {
    const u64 r1 = shoup_lazy(a.hi, p.r64, p.r64s, p.q, p.qn);
    const u64 r2 = a.lo - mulhi(a.lo, p.ones) * p.q;
    return red4(r1 + r2, p.q, p.q2);
}
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const PrimeConst &p) {
    Acc t;
    t.lo = a * b;
    t.hi = mulhi(a, b);
    return acc_reduce(t, p);
}
// x mod q for any x < 2^64
__device__ __forceinline__ u64 reduce_any(u64 x, const PrimeConst &p) {
    return red2(x - mulhi(x, p.ones) * p.q, p.q);
}
// centered lift of x in [0, qf) to modulus p: x > (qf-1)/2 stands for x - qf
__device__ __forceinline__ u64 lift_centered(u64 x, u64 qf, u64 qf_mod, const PrimeConst &p) {
    const u64 y = reduce_any(x, p);
    return x > (qf >> 1) ? sub_mod(y, qf_mod, p.q) : y;
}

// ---------------------------------------------------------------- exact FP64 modular arithmetic
// For a prime q < 2^41 residues are kept as integer-valued doubles. With fl(1/q) = qinv,
//   ph = fl(y w), pl = fma(y, w, -ph) (the exact rounding error), qh = rint(ph * qinv),
//   r = fma(-qh, q, ph) + pl
// gives r = y w - qh q exactly, with |r| <= 0.52 q whenever |y| < 2^45 and 0 <= w < q: the
// quotient estimate is within 0.52 of y w / q, ph - qh q = r - pl has magnitude below 2^53 and is
// produced exactly by the fma, and the final sum of two integers below 2^53 is exact. All FP64
// instructions issue at the full VALU rate on gfx950, so a product costs 5 instructions instead
// of the ~16 of the 64-bit integer form.
__device__ __forceinline__ double fp_mul(double y, double w, double q, double qinv) {
    const double ph = y * w;
    const double pl = __fma_rn(y, w, -ph);
    const double qh = rint(ph * qinv);
    return __fma_rn(-qh, q, ph) + pl;
}
// v - rint(v / q) q: |result| <= 0.51 q for integer-valued |v| < 2^51
__device__ __forceinline__ double fp_center(double v, double q, double qinv) {
    return __fma_rn(-rint(v * qinv), q, v);
}
// Integer-valued doubles in [0, 2^52) and u64 words below 2^52 convert through the bit pattern of
// 2^52 + x, whose exponent is fixed: two instructions each way instead of a library conversion.
__device__ __forceinline__ u64 fp_to_u64(double v, double q, double qinv) {
    double r = fp_center(v, q, qinv);
    r = r < 0.0 ? r + q : r;
    return (u64)__double_as_longlong(r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}
__device__ __forceinline__ double u64_to_fp(u64 x) {      // x < 2^52
    return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - 4503599627370496.0;
}

// Index gathered by the automorphism X -> X^g in bit-reversed NTT order:
// out[i] = in[brv((g (2 brv(i) + 1) mod 2N - 1) / 2)].
__device__ __forceinline__ int galois_src(int i, u64 g, int logn) {
    const unsigned n = 1u << logn;
    const unsigned e = (__brev((unsigned)i) >> (32 - logn));
    const unsigned t = (unsigned)((g * (2ull * e + 1)) & (2ull * n - 1));
    return (int)(__brev((t - 1) >> 1) >> (32 - logn));
}

// ---------------------------------------------------------------- buffer loads and stores
// A raw buffer resource over `bytes` bytes from `base` (scalar registers when base is uniform):
// a load or store then addresses base + voffset (a per-lane 32-bit byte offset) + soffset (a
// uniform one) with no address arithmetic on the vector ALU. Accesses at or past `bytes` read 0
// and write nothing. Third descriptor word 0x00020000: raw 32-bit data, as for every gfx9 part.
// Stores are non-temporal: their data (rotated ciphertexts, read back by a later kernel) would
// otherwise displace the digit words that the key product's workgroups share through L2.
typedef __amdgpu_buffer_rsrc_t BufRsrc;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ BufRsrc buf_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ u64 buf_load(BufRsrc r, int voffset, int soffset) {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voffset, soffset, 0);
    return ((u64)v.y << 32) | v.x;
}
__device__ __forceinline__ void buf_store(u64 x, BufRsrc r, int voffset, int soffset) {
    u32x2 v;
    v.x = (unsigned)x;
    v.y = (unsigned)(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voffset, soffset, 2);    // nt: streamed, not kept in L2
}

// ---------------------------------------------------------------- NTT engine
template <int LOGN>
struct Geo {
    static constexpr int N = 1 << LOGN;
    static constexpr int T = N / 16;   // threads per residue
};

__device__ __forceinline__ int lds_idx(int j) { return j + (j >> 5); }

template <int LOGN>
constexpr int lds_words() { return (1 << LOGN) + ((1 << LOGN) >> 5); }

// Element index of slot (g, e) of a pass over bits [LO, LO + RB): e supplies those bits, the
// group g and the thread the others. Workgroup mapping (WV = false): rest = g T + tid spans the
// whole residue. Wave-local mapping (WV = true), for passes below bit 10 after the first one: wave
// w = tid / 64 keeps the 1024 elements [1024 w, 1024 w + 1024), the bits of its lane and of g
// filling the rest, so the pass and its LDS exchange involve that wave alone (after the first pass
// the transform splits into independent sub-transforms over the lower bits).
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ int pass_rest(int g, int tid) {
    return WV ? (g << 6) | (tid & 63) : g * Geo<LOGN>::T + tid;
}
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ int pass_index(int g, int e, int tid) {
    const int rest = pass_rest<LOGN, LO, RB, WV>(g, tid);
    const int idx = ((rest >> LO) << (LO + RB)) | (e << LO) | (rest & ((1 << LO) - 1));
    return WV ? ((tid >> 6) << 10) | idx : idx;
}
// index >> (LO + RB) of the elements of group g (the twiddles of every stage of the pass follow
// from it): uniform across a wave when LO >= 6
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ int pass_hi(int g, int tid) {
    const int hi = pass_rest<LOGN, LO, RB, WV>(g, tid) >> LO;
    return WV ? ((tid >> 6) << (10 - LO - RB)) | hi : hi;
}

// Order the LDS accesses of one wave: its lanes' writes before its later reads (a wave's LDS
// operations execute in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Element j of the wave-local output / input layout: wave w's 1024 elements, 64 consecutive per
// value slot e (coalesced loads and stores).
__device__ __forceinline__ int wave_elem(int tid, int e) { return ((tid >> 6) << 10) | (e << 6) | (tid & 63); }

template <int LOGN, int LO, int RB, bool WV = false, typename T>
__device__ __forceinline__ void to_lds(const T (&v)[16], T *lds, int tid) {
    constexpr int R = 1 << RB, G = 16 / R;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < R; ++e) lds[lds_idx(pass_index<LOGN, LO, RB, WV>(g, e, tid))] = v[g * R + e];
}

template <int LOGN, int LO, int RB, bool WV = false, typename T>
__device__ __forceinline__ void from_lds(T (&v)[16], const T *lds, int tid) {
    constexpr int R = 1 << RB, G = 16 / R;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int e = 0; e < R; ++e) v[g * R + e] = lds[lds_idx(pass_index<LOGN, LO, RB, WV>(g, e, tid))];
}

// Cooley-Tukey stages over bits LO+RB-1 .. LO. Values enter and leave in [0, 4q).
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ void fwd_pass(u64 (&v)[16], int tid, const u64 *__restrict__ tw,
                                         const u64 *__restrict__ tws, u64 q, u64 q2, u64 qn, u64 nq2) {
    constexpr int R = 1 << RB, G = 16 / R, N = Geo<LOGN>::N;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // for LO >= 6 the 64 lanes of a wave share hi: make that visible so twiddles use scalar loads
        const int hi = LO >= 6 ? __builtin_amdgcn_readfirstlane(pass_hi<LOGN, LO, RB, WV>(g, tid))
                               : pass_hi<LOGN, LO, RB, WV>(g, tid);
#pragma unroll
        for (int sb = RB - 1; sb >= 0; --sb) {
            const int b = LO + sb, half = 1 << sb;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                if (e & half) continue;
                const int widx = (N >> (b + 1)) + ((hi << (RB - 1 - sb)) | (e >> (sb + 1)));
                const u64 w = tw[widx], ws = tws[widx];
                const u64 x = csub(v[g * R + e], nq2);
                const u64 t = shoup_lazy(v[g * R + e + half], w, ws, q, qn);
                v[g * R + e] = x + t;
                v[g * R + e + half] = x + q2 - t;
            }
        }
    }
}

// Gentleman-Sande stages over bits LO .. LO+RB-1. Values enter and leave in [0, 2q).
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ void inv_pass(u64 (&v)[16], int tid, const u64 *__restrict__ tw,
                                         const u64 *__restrict__ tws, u64 q, u64 q2, u64 qn, u64 nq2) {
    constexpr int R = 1 << RB, G = 16 / R, N = Geo<LOGN>::N;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // for LO >= 6 the 64 lanes of a wave share hi: make that visible so twiddles use scalar loads
        const int hi = LO >= 6 ? __builtin_amdgcn_readfirstlane(pass_hi<LOGN, LO, RB, WV>(g, tid))
                               : pass_hi<LOGN, LO, RB, WV>(g, tid);
#pragma unroll
        for (int sb = 0; sb < RB; ++sb) {
            const int b = LO + sb, half = 1 << sb;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                if (e & half) continue;
                const int widx = (N >> (b + 1)) + ((hi << (RB - 1 - sb)) | (e >> (sb + 1)));
                const u64 w = tw[widx], ws = tws[widx];
                const u64 x = v[g * R + e], y = v[g * R + e + half];
                v[g * R + e] = csub(x + y, nq2);
                v[g * R + e + half] = shoup_lazy(x + q2 - y, w, ws, q, qn);
            }
        }
    }
}

// FP64 Cooley-Tukey stages (prime < 2^41): t = w y with |t| <= 0.52 q, outputs x + t and x - t.
// From canonical inputs the magnitude stays below (1 + 0.52 s) q after s stages (< 2^45 after 14),
// so no intermediate reduction is needed.
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ void fwd_pass_fp(double (&v)[16], int tid, const double *__restrict__ tw, double q,
                                            double qinv) {
    constexpr int R = 1 << RB, G = 16 / R, N = Geo<LOGN>::N;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // for LO >= 6 the 64 lanes of a wave share hi: make that visible so twiddles use scalar loads
        const int hi = LO >= 6 ? __builtin_amdgcn_readfirstlane(pass_hi<LOGN, LO, RB, WV>(g, tid))
                               : pass_hi<LOGN, LO, RB, WV>(g, tid);
#pragma unroll
        for (int sb = RB - 1; sb >= 0; --sb) {
            const int b = LO + sb, half = 1 << sb;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                if (e & half) continue;
                const int widx = (N >> (b + 1)) + ((hi << (RB - 1 - sb)) | (e >> (sb + 1)));
                const double t = fp_mul(v[g * R + e + half], tw[widx], q, qinv);
                const double x = v[g * R + e];
                v[g * R + e] = x + t;
                v[g * R + e + half] = x - t;
            }
        }
    }
}

// FP64 Gentleman-Sande stages: x + y and (x - y) w. Sums double per stage, so every value is
// centered (|v| <= 0.51 q) at the end of each pass: within a pass of at most 4 stages magnitudes
// stay below 16 q < 2^45.
template <int LOGN, int LO, int RB, bool WV = false>
__device__ __forceinline__ void inv_pass_fp(double (&v)[16], int tid, const double *__restrict__ tw, double q,
                                            double qinv) {
    constexpr int R = 1 << RB, G = 16 / R, N = Geo<LOGN>::N;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // for LO >= 6 the 64 lanes of a wave share hi: make that visible so twiddles use scalar loads
        const int hi = LO >= 6 ? __builtin_amdgcn_readfirstlane(pass_hi<LOGN, LO, RB, WV>(g, tid))
                               : pass_hi<LOGN, LO, RB, WV>(g, tid);
#pragma unroll
        for (int sb = 0; sb < RB; ++sb) {
            const int b = LO + sb, half = 1 << sb;
#pragma unroll
            for (int e = 0; e < R; ++e) {
                if (e & half) continue;
                const int widx = (N >> (b + 1)) + ((hi << (RB - 1 - sb)) | (e >> (sb + 1)));
                const double x = v[g * R + e], y = v[g * R + e + half];
                v[g * R + e] = x + y;
                v[g * R + e + half] = fp_mul(x - y, tw[widx], q, qinv);
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = fp_center(v[e], q, qinv);
}

// Pass plans (bit ranges, lowest bit first for each pass):
//   N = 2^12: [8,12) [4,8) [0,4)      N = 2^13: [9,13) [6,9) [3,6) [0,3)
//   N = 2^14: [10,14) [6,10) [3,6) [0,3)
// The top pass spans the whole residue (workgroup mapping: thread tid holds elements tid + T e)
// and is the only one that needs a workgroup barrier; the passes below it are wave-local (see
// pass_index), so each wave runs them on its own 1024 elements with no barrier, overlapping the
// other waves' exchanges. The arithmetic of every butterfly is the same whatever the mapping.
//
// Forward: v holds elements j = tid + T e on entry; on exit the transformed residue is in LDS
// (lds_idx(j)), values in [0, 4q) (integer) or |v| < 2^45 (FP64), and wave w's elements
// [1024 w, 1024 w + 1024) are visible to wave w (read them through wave_elem).
// Inverse: wave w's elements are in LDS (written by the wave itself, then wave_sync) on entry; on
// exit v holds elements j = tid + T e, values in [0, 2q) (integer) or centered (FP64), not yet
// multiplied by N^{-1}.
// The passes below the top one, wave-local: `lt` is the thread index used for the LDS mapping
// (the workgroup's tid with a residue-sized LDS, or the lane with one wave's 1024-element region),
// the pass functor carries the tid used for the twiddles.
template <int LOGN, typename T, typename Pass>
__device__ __forceinline__ void fwd_sub_plan(T (&v)[16], T *lds, int lt, Pass &&pass) {
    if constexpr (LOGN == 12) {
        from_lds<12, 4, 4, true>(v, lds, lt);
        pass(std::integral_constant<int, 4>{}, std::integral_constant<int, 4>{}, std::true_type{});
        to_lds<12, 4, 4, true>(v, lds, lt); wave_sync();
        from_lds<12, 0, 4, true>(v, lds, lt);
        pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 4>{}, std::true_type{});
        to_lds<12, 0, 4, true>(v, lds, lt); wave_sync();
    } else if constexpr (LOGN == 13) {
        from_lds<13, 6, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 6>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<13, 6, 3, true>(v, lds, lt); wave_sync();
        from_lds<13, 3, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<13, 3, 3, true>(v, lds, lt); wave_sync();
        from_lds<13, 0, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<13, 0, 3, true>(v, lds, lt); wave_sync();
    } else {
        static_assert(LOGN == 14, "unsupported ring degree");
        from_lds<14, 6, 4, true>(v, lds, lt);
        pass(std::integral_constant<int, 6>{}, std::integral_constant<int, 4>{}, std::true_type{});
        to_lds<14, 6, 4, true>(v, lds, lt); wave_sync();
        from_lds<14, 3, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<14, 3, 3, true>(v, lds, lt); wave_sync();
        from_lds<14, 0, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<14, 0, 3, true>(v, lds, lt); wave_sync();
    }
}

template <int LOGN, typename T, typename Pass>
__device__ __forceinline__ void inv_sub_plan(T (&v)[16], T *lds, int lt, Pass &&pass) {
    if constexpr (LOGN == 12) {
        from_lds<12, 0, 4, true>(v, lds, lt);
        pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 4>{}, std::true_type{});
        to_lds<12, 0, 4, true>(v, lds, lt); wave_sync();
        from_lds<12, 4, 4, true>(v, lds, lt);
        pass(std::integral_constant<int, 4>{}, std::integral_constant<int, 4>{}, std::true_type{});
        to_lds<12, 4, 4, true>(v, lds, lt); wave_sync();
    } else if constexpr (LOGN == 13) {
        from_lds<13, 0, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<13, 0, 3, true>(v, lds, lt); wave_sync();
        from_lds<13, 3, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<13, 3, 3, true>(v, lds, lt); wave_sync();
        from_lds<13, 6, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 6>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<13, 6, 3, true>(v, lds, lt); wave_sync();
    } else {
        static_assert(LOGN == 14, "unsupported ring degree");
        from_lds<14, 0, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 0>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<14, 0, 3, true>(v, lds, lt); wave_sync();
        from_lds<14, 3, 3, true>(v, lds, lt);
        pass(std::integral_constant<int, 3>{}, std::integral_constant<int, 3>{}, std::true_type{});
        to_lds<14, 3, 3, true>(v, lds, lt); wave_sync();
        from_lds<14, 6, 4, true>(v, lds, lt);
        pass(std::integral_constant<int, 6>{}, std::integral_constant<int, 4>{}, std::true_type{});
        to_lds<14, 6, 4, true>(v, lds, lt); wave_sync();
    }
}

// The whole transform in one workgroup: the top pass over bits [LOGN - 4, LOGN), one workgroup
// exchange, then the wave-local passes.
template <int LOGN, typename T, typename Pass>
__device__ __forceinline__ void fwd_plan(T (&v)[16], T *lds, int tid, Pass &&pass) {
    constexpr int TOP = LOGN - 4;
    pass(std::integral_constant<int, TOP>{}, std::integral_constant<int, 4>{}, std::false_type{});
    to_lds<LOGN, TOP, 4>(v, lds, tid);
    __syncthreads();
    fwd_sub_plan<LOGN>(v, lds, tid, pass);
}

template <int LOGN, typename T, typename Pass>
__device__ __forceinline__ void inv_plan(T (&v)[16], T *lds, int tid, Pass &&pass) {
    constexpr int TOP = LOGN - 4;
    inv_sub_plan<LOGN>(v, lds, tid, pass);
    __syncthreads();
    from_lds<LOGN, TOP, 4>(v, lds, tid);
    pass(std::integral_constant<int, TOP>{}, std::integral_constant<int, 4>{}, std::false_type{});
}

template <int LOGN>
__device__ __forceinline__ void ntt_fwd_core_fp(double (&v)[16], double *lds, int tid, const double *tw,
                                                double q, double qinv) {
    fwd_plan<LOGN>(v, lds, tid, [&](auto lo, auto rb, auto wv) {
        fwd_pass_fp<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, q, qinv);
    });
}

template <int LOGN>
__device__ __forceinline__ void ntt_inv_core_fp(double (&v)[16], double *lds, int tid, const double *tw,
                                                double q, double qinv) {
    inv_plan<LOGN>(v, lds, tid, [&](auto lo, auto rb, auto wv) {
        inv_pass_fp<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, q, qinv);
    });
}

template <int LOGN>
__device__ __forceinline__ void ntt_fwd_core(u64 (&v)[16], u64 *lds, int tid, const u64 *tw,
                                             const u64 *tws, const PrimeConst &pc) {
    const u64 q = pc.q, q2 = pc.q2, qn = pc.qn, nq2 = pc.nq2;
    fwd_plan<LOGN>(v, lds, tid, [&](auto lo, auto rb, auto wv) {
        fwd_pass<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, tws, q, q2, qn, nq2);
    });
}

template <int LOGN>
__device__ __forceinline__ void ntt_inv_core(u64 (&v)[16], u64 *lds, int tid, const u64 *tw,
                                             const u64 *tws, const PrimeConst &pc) {
    const u64 q = pc.q, q2 = pc.q2, qn = pc.qn, nq2 = pc.nq2;
    inv_plan<LOGN>(v, lds, tid, [&](auto lo, auto rb, auto wv) {
        inv_pass<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, tws, q, q2, qn, nq2);
    });
}

__device__ __forceinline__ long res_offset(const ResMap &m, int r) {
    const int e = r % m.per, t = r / m.per;
    return m.off + (long)(t / m.ngrp) * m.ostride + (long)(t % m.ngrp) * m.gstride + e;
}

// x, opaque to the compiler: index arithmetic derived from it (inside a loop iteration, or per
// loaded element) is redone where it is used rather than hoisted and kept in registers.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// ---------------------------------------------------------------- NTT kernels
// Every NTT-bearing kernel picks the arithmetic per workgroup from its prime (uniform branch):
// FP64 for primes below 2^41, 64-bit integer otherwise. Inputs and outputs are canonical residues
// in [0, q) either way, so the results are the same integers.

// Forward transform of canonical values v[e] (element tid + T e) held in registers; the result is
// left in LDS (as doubles for an FP64 prime, as lazy [0, 4q) integers otherwise), wave w's part
// (elements wave_elem(tid, e)) visible to wave w. Returns fp.
template <int LOGN>
__device__ __forceinline__ bool fwd_transform(u64 (&v)[16], u64 *lds, int tid, const Tables &tab, int pi,
                                              const PrimeConst &p) {
    constexpr int N = Geo<LOGN>::N;
    if (p.fp) {
        double d[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = u64_to_fp(v[e]);
        ntt_fwd_core_fp<LOGN>(d, reinterpret_cast<double *>(lds), tid,
                              reinterpret_cast<const double *>(tab.tws + (long)pi * N), p.qd, p.qinv);
        return true;
    }
    ntt_fwd_core<LOGN>(v, lds, tid, tab.tw + (long)pi * N, tab.tws + (long)pi * N, p);
    return false;
}

// Canonical value of output element j of fwd_transform.
__device__ __forceinline__ u64 fwd_result(const u64 *lds, int j, bool fp, const PrimeConst &p) {
    if (fp) return fp_to_u64(reinterpret_cast<const double *>(lds)[lds_idx(j)], p.qd, p.qinv);
    return red4(lds[lds_idx(j)], p.q, p.q2);
}

template <int LOGN>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_ntt_fwd(const u64 *__restrict__ in, ResMap imap, u64 *__restrict__ out, ResMap omap, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T;
    const int tid = threadIdx.x, r = blockIdx.x;
    const int pi = imap.prime[r % imap.per];
    const PrimeConst p = tab.pc[pi];
    const u64 *src = in + res_offset(imap, r) * N;
    u64 *dst = out + res_offset(omap, r) * N;
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = src[tid + T * e];
    const bool fp = fwd_transform<LOGN>(v, lds, tid, tab, pi, p);
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[wave_elem(tid, e)] = fwd_result(lds, wave_elem(tid, e), fp, p);
}

template <int LOGN>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_ntt_inv(const u64 *__restrict__ in, ResMap imap, u64 *__restrict__ out, ResMap omap, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T;
    const int tid = threadIdx.x, r = blockIdx.x;
    const int pi = imap.prime[r % imap.per];
    const PrimeConst p = tab.pc[pi];
    const u64 *src = in + res_offset(imap, r) * N;
    u64 *dst = out + res_offset(omap, r) * N;
    if (p.fp) {
        double *dl = reinterpret_cast<double *>(lds);
#pragma unroll
        for (int e = 0; e < 16; ++e) dl[lds_idx(wave_elem(tid, e))] = u64_to_fp(src[wave_elem(tid, e)]);
        wave_sync();
        double d[16];
        ntt_inv_core_fp<LOGN>(d, dl, tid, reinterpret_cast<const double *>(tab.itws + (long)pi * N), p.qd, p.qinv);
#pragma unroll
        for (int e = 0; e < 16; ++e) dst[tid + T * e] = fp_to_u64(fp_mul(d[e], p.ninvd, p.qd, p.qinv), p.qd, p.qinv);
        return;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[lds_idx(wave_elem(tid, e))] = src[wave_elem(tid, e)];
    wave_sync();
    u64 v[16];
    ntt_inv_core<LOGN>(v, lds, tid, tab.itw + (long)pi * N, tab.itws + (long)pi * N, p);
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[tid + T * e] = red2(shoup_lazy(v[e], p.ninv, p.ninvs, p.q, p.qn), p.q);
}

// ModUp: coef is dense [G][k][N] coefficient form; digit j of group g is lifted (centered) from
// q_j to every target t in 0..k (t = k is the special prime) and transformed:
// digits[g][j][t] (NTT form). The diagonal t = j is the input residue itself (the lift from q_j to
// q_j is the identity), copied from d (NTT form, residue g k + j of dmap). One workgroup per
// (g, j, t). The digits are stored non-temporally: the key product reads them after every
// workgroup here has finished, so keeping them in L2 only displaces the coefficients this kernel
// re-reads (the MAC's outputs are stored the same way for the same reason).
// Targets with an FP64 prime hold the bit patterns of FP64 values congruent to the digit, of
// magnitude below 2^45 (the forward transform's output as it stands, or the copied residue): the
// key product, their only reader, multiplies them as they are.
template <int LOGN>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_modup(const u64 *__restrict__ coef, const u64 *__restrict__ d, ResMap dmap, u64 *__restrict__ digits, int k,
        int nq, int units, int xcd_order, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T;
    const int tid = opaque(threadIdx.x);
    int t, gj;                                // gj = g * k + j, the digit; t, its target
    if (xcd_order) {
        // the k + 1 targets of a digit run back to back on one XCD (workgroups are dealt to the 8
        // XCDs in turn), so its L2 serves the k re-reads of the digit
        const int loc = blockIdx.x >> 3;
        t = loc % (k + 1);
        gj = (loc / (k + 1)) * 8 + (blockIdx.x & 7);
        if (gj >= units) return;
    } else {
        t = blockIdx.x % (k + 1);
        gj = blockIdx.x / (k + 1);
    }
    const int j = gj % k;
    u64 *dst = digits + ((long)gj * (k + 1) + t) * N;
    if (t == j) {
        const u64 *src = d + res_offset(dmap, gj) * N;
        if (tab.pc[t].fp) {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                dst[tid + T * e] = (u64)__double_as_longlong(u64_to_fp(src[tid + T * e]));
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) dst[tid + T * e] = src[tid + T * e];
        }
        return;
    }
    const int pt = t < k ? t : nq;
    const PrimeConst p = tab.pc[pt];
    const u64 qj = tab.pc[j].q;
    const u64 qj_mod = tab.cross[pt * kMaxMods + j].qj_mod_qi;
    const u64 *src = coef + (long)gj * N;
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = lift_centered(src[tid + T * e], qj, qj_mod, p);
    if (fwd_transform<LOGN>(v, lds, tid, tab, pt, p)) {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            __builtin_nontemporal_store(lds[lds_idx(wave_elem(tid, e))], &dst[wave_elem(tid, e)]);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e)
            __builtin_nontemporal_store(fwd_result(lds, wave_elem(tid, e), false, p), &dst[wave_elem(tid, e)]);
    }
}

// Drop the last modulus of each group (ModDown when it is P, rescale when it is q_k):
//   out[g][i] = (x[g][i] - NTT_i(lift(last[g]))) * m_last^{-1} mod q_i  (+ addend)
// x: [G][k+1][N] NTT form (only i < k read), group g at xm.off + (g / xm.R) xm.sb + (g % xm.R) xm.sr;
// last: dense [G][N] coefficient form mod m_last; out: [G][k][N]. Groups are (b, r, c) with G = B R 2; the addend for polynomial c (if bit c of
// add_mask) is read at add + b sb + r sr + c sc + i N, gathered through sigma_{gal[r]}.
template <int LOGN>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_drop(const u64 *__restrict__ x, GrpMap xm, const u64 *__restrict__ last, u64 *__restrict__ out, int k,
       int drop, int groups, int xcd_order, DropAdd add, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T;
    const int tid = opaque(threadIdx.x);
    int i, grp;
    if (xcd_order) {
        // the k primes of a group run back to back on one XCD, which then reads `last` once
        const int loc = blockIdx.x >> 3;
        i = loc % k;
        grp = (loc / k) * 8 + (blockIdx.x & 7);
        if (grp >= groups) return;
    } else {
        i = blockIdx.x % k;
        grp = blockIdx.x / k;
    }
    const PrimeConst p = tab.pc[i];
    const u64 qd = tab.pc[drop].q;
    const CrossConst cc = tab.cross[i * kMaxMods + drop];
    const u64 *src = last + (long)grp * N;
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = lift_centered(src[tid + T * e], qd, cc.qj_mod_qi, p);
    const bool fp = fwd_transform<LOGN>(v, lds, tid, tab, i, p);
    const u64 *xi = x + xm.off + (long)(grp / xm.R) * xm.sb + (long)(grp % xm.R) * xm.sr + (long)i * N;
    u64 *dst = out + ((long)grp * k + i) * N;
    const int c = grp & 1, r = (grp >> 1) % add.R, b = (grp >> 1) / add.R;
    const bool has_add = (add.mask >> c) & 1;
    const u64 *ap = has_add ? add.base + b * add.sb + r * add.sr + c * add.sc + (long)i * N : nullptr;
    const u64 g = add.gal[r];
    if (fp) {
        const double *dl = reinterpret_cast<const double *>(lds);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int jj = wave_elem(tid, e);
            double val = fp_mul(u64_to_fp(xi[jj]) - dl[lds_idx(jj)], cc.invd, p.qd, p.qinv);
            if (has_add) val += u64_to_fp(ap[g == 1 ? jj : galois_src(jj, g, LOGN)]);
            dst[jj] = fp_to_u64(val, p.qd, p.qinv);
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int jj = wave_elem(tid, e);
        const u64 ext = red4(lds[lds_idx(jj)], p.q, p.q2);
        u64 val = red2(shoup_lazy(sub_mod(xi[jj], ext, p.q), cc.inv, cc.invs, p.q, p.qn), p.q);
        if (has_add) val = add_mod(val, ap[g == 1 ? jj : galois_src(jj, g, LOGN)], p.q);
        dst[jj] = val;
    }
}

// ---------------------------------------------------------------- split transforms (few residues)
// A launch of fewer residue transforms than CUs leaves most of the GPU idle, and one transform
// takes a single CU tens of microseconds. Split, a transform runs as two launches of N / 1024
// single-wave workgroups each: for the forward transform the top pass (each thread's 16 values
// at stride T, as in the one-workgroup form), its result through a buffer (kept in L2), then each
// wave's 1024 elements through the wave-local passes; the inverse the other way round. Every
// butterfly is the one of the one-workgroup form, so the residues are the same. The operations
// around the transform (lift on the load, combine on the store) come from an Op:
//   prime(r)      prime-table index of residue r of the launch
//   copy_only(r)  residue r is a plain copy (copy(r, j, tab) for element j), no transform
//   load(r, j, p, tab)                          input of element j, canonical mod p: the word
//                                               fetch(r, j) brought to p by prep(r, x, p, tab)
//   store_fwd(r, j, x, fp, p, tab)              forward output: x as the LDS of the one-workgroup
//                                               form holds it (double bits for an FP64 prime)
//   store_inv(r, j, x, p) / store_inv_fp(r, j, d, p)   inverse output before the N^{-1} factor
struct OpNtt {
    const u64 *in;
    ResMap imap;
    u64 *out;
    ResMap omap;
    int logn;
    __device__ int prime(int r) const { return imap.prime[r % imap.per]; }
    __device__ bool copy_only(int) const { return false; }
    __device__ void copy(int, int, const Tables &) const {}
    __device__ u64 fetch(int r, int j) const { return in[(res_offset(imap, r) << logn) + j]; }
    __device__ u64 prep(int, u64 x, const PrimeConst &, const Tables &) const { return x; }
    __device__ u64 load(int r, int j, const PrimeConst &p, const Tables &tab) const { return prep(r, fetch(r, j), p, tab); }
    __device__ void store_fwd(int r, int j, u64 x, bool fp, const PrimeConst &p, const Tables &) const {
        out[(res_offset(omap, r) << logn) + j] =
            fp ? fp_to_u64(__longlong_as_double((long long)x), p.qd, p.qinv) : red4(x, p.q, p.q2);
    }
    __device__ void store_inv(int r, int j, u64 x, const PrimeConst &p) const {
        out[(res_offset(omap, r) << logn) + j] = red2(shoup_lazy(x, p.ninv, p.ninvs, p.q, p.qn), p.q);
    }
    __device__ void store_inv_fp(int r, int j, double d, const PrimeConst &p) const {
        out[(res_offset(omap, r) << logn) + j] = fp_to_u64(fp_mul(d, p.ninvd, p.qd, p.qinv), p.qd, p.qinv);
    }
};

// ModUp (see k_modup), residues numbered r = gj (k + 1) + t.
struct OpModup {
    const u64 *coef, *d;
    ResMap dmap;
    u64 *digits;
    int k, nq, logn;
    __device__ int prime(int r) const { const int t = r % (k + 1); return t < k ? t : nq; }
    __device__ bool copy_only(int r) const { return r % (k + 1) == (r / (k + 1)) % k; }
    __device__ void copy(int r, int j, const Tables &tab) const {
        const int t = r % (k + 1), gj = r / (k + 1);
        const u64 x = d[(res_offset(dmap, gj) << logn) + j];
        digits[(((long)gj * (k + 1) + t) << logn) + j] = tab.pc[t].fp ? (u64)__double_as_longlong(u64_to_fp(x)) : x;
    }
    __device__ u64 fetch(int r, int j) const { return coef[((long)(r / (k + 1)) << logn) + j]; }
    __device__ u64 prep(int r, u64 x, const PrimeConst &p, const Tables &tab) const {
        const int t = r % (k + 1), j0 = (r / (k + 1)) % k, pt = t < k ? t : nq;
        return lift_centered(x, tab.pc[j0].q, tab.cross[pt * kMaxMods + j0].qj_mod_qi, p);
    }
    __device__ u64 load(int r, int j, const PrimeConst &p, const Tables &tab) const { return prep(r, fetch(r, j), p, tab); }
    __device__ void store_fwd(int r, int j, u64 x, bool fp, const PrimeConst &p, const Tables &) const {
        const int t = r % (k + 1), gj = r / (k + 1);
        __builtin_nontemporal_store(fp ? x : red4(x, p.q, p.q2), &digits[(((long)gj * (k + 1) + t) << logn) + j]);
    }
    __device__ void store_inv(int, int, u64, const PrimeConst &) const {}
    __device__ void store_inv_fp(int, int, double, const PrimeConst &) const {}
};

// Drop the last modulus (see k_drop), residues numbered r = grp k + i.
struct OpDrop {
    const u64 *x;
    GrpMap xm;
    const u64 *last;
    u64 *out;
    int k, drop, logn;
    DropAdd add;
    __device__ int prime(int r) const { return r % k; }
    __device__ bool copy_only(int) const { return false; }
    __device__ void copy(int, int, const Tables &) const {}
    __device__ u64 fetch(int r, int j) const { return last[((long)(r / k) << logn) + j]; }
    __device__ u64 prep(int r, u64 x, const PrimeConst &p, const Tables &tab) const {
        return lift_centered(x, tab.pc[drop].q, tab.cross[(r % k) * kMaxMods + drop].qj_mod_qi, p);
    }
    __device__ u64 load(int r, int j, const PrimeConst &p, const Tables &tab) const { return prep(r, fetch(r, j), p, tab); }
    __device__ void store_fwd(int r, int j, u64 v, bool fp, const PrimeConst &p, const Tables &tab) const {
        const int i = r % k, grp = r / k;
        const long N = 1L << logn;
        const CrossConst cc = tab.cross[i * kMaxMods + drop];
        const u64 xv = x[xm.off + (long)(grp / xm.R) * xm.sb + (long)(grp % xm.R) * xm.sr + (long)i * N + j];
        const int c = grp & 1, rr = (grp >> 1) % add.R, b = (grp >> 1) / add.R;
        const bool has_add = (add.mask >> c) & 1;
        const u64 g = add.gal[rr];
        const u64 av = has_add ? add.base[b * add.sb + rr * add.sr + c * add.sc + (long)i * N +
                                          (g == 1 ? j : galois_src(j, g, logn))] : 0;
        u64 *dst = out + ((long)grp * k + i) * N + j;
        if (fp) {
            double val = fp_mul(u64_to_fp(xv) - __longlong_as_double((long long)v), cc.invd, p.qd, p.qinv);
            if (has_add) val += u64_to_fp(av);
            *dst = fp_to_u64(val, p.qd, p.qinv);
            return;
        }
        const u64 ext = red4(v, p.q, p.q2);
        u64 val = red2(shoup_lazy(sub_mod(xv, ext, p.q), cc.inv, cc.invs, p.q, p.qn), p.q);
        if (has_add) val = add_mod(val, av, p.q);
        *dst = val;
    }
    __device__ void store_inv(int, int, u64, const PrimeConst &) const {}
    __device__ void store_inv_fp(int, int, double, const PrimeConst &) const {}
};

// ModDown by P followed by the rescale by q_l, l = kl (the last prime of Q), in one forward pass
// (hybrid key switch, then the rescale, Section 2). With c_P the coefficients of the P row and
// y_l those of the ModDown result's row l, the two steps give, for i < l,
//   out_i = ((x_i - NTT([c_P]_i)) P^-1 + a_i - NTT([y_l]_i)) q_l^-1
//         = ((x_i - NTT([c_P]_i + P [y_l]_i)) P^-1 + a_i) q_l^-1          (NTT is linear mod q_i)
// ([c]_i the centred lift of c into q_i), and y_l = (c_l - [c_P]_l) P^-1 mod q_l with c_l the
// coefficients of row l of x: when the addend a is present its row l has been added to x's as
// P a_l beforehand (see k_fold_last), which puts a_l into y_l. So the forward transforms take
// [c_P]_i + P [y_l]_i (computed from the two coefficient rows by load) and the combine multiplies
// by P^-1 and q_l^-1 in turn: the residues of the two steps, with one inverse transform more and
// the k forward transforms of the ModDown's own pass fewer. Residues r = g kl + i.
struct OpDropRescale {
    const u64 *x;        // group g, row t at x + g xs + t N (rows 0..kl over Q, kl + 1 the P row)
    long xs;
    const u64 *coef;     // [groups][2][N]: inverse transforms of row kl (mod q_kl) and of the P row
    u64 *out;            // [groups][kl][N]
    int kl, np, logn;
    DropAdd add;         // R = 1, no rotation: polynomial c of group g = 2 b + c adds base + b sb + c sc
    __device__ int prime(int r) const { return r % kl; }
    __device__ bool copy_only(int) const { return false; }
    __device__ void copy(int, int, const Tables &) const {}
    __device__ u64 fetch(int r, int j) const { return coef[((long)(r / kl) * 2 << logn) + j]; }
    __device__ u64 prep(int, u64 x, const PrimeConst &, const Tables &) const { return x; }
    __device__ u64 load(int r, int j, const PrimeConst &p, const Tables &tab) const {
        const long g = r / kl;
        return combine(r, coef[(g * 2 << logn) + j], coef[((g * 2 + 1) << logn) + j], p, tab);
    }
    // [c_P]_i + P [y_l]_i mod q_i from the coefficients cl (mod q_kl) and cp (mod P)
    __device__ u64 combine(int r, u64 cl, u64 cp, const PrimeConst &p, const Tables &tab) const {
        const int i = r % kl;
        const PrimeConst pl = tab.pc[kl];
        const u64 P = tab.pc[np].q;
        const CrossConst lp = tab.cross[kl * kMaxMods + np];
        const u64 yl = red2(shoup_lazy(sub_mod(cl, lift_centered(cp, P, lp.qj_mod_qi, pl), pl.q), lp.inv, lp.invs,
                                       pl.q, pl.qn), pl.q);
        const CrossConst ip = tab.cross[i * kMaxMods + np];
        const u64 a = lift_centered(cp, P, ip.qj_mod_qi, p);
        const u64 b = lift_centered(yl, pl.q, tab.cross[i * kMaxMods + kl].qj_mod_qi, p);
        return add_mod(a, mul_mod(b, ip.qj_mod_qi, p), p.q);
    }
    __device__ void store_fwd(int r, int j, u64 v, bool fp, const PrimeConst &p, const Tables &tab) const {
        const int i = r % kl, grp = r / kl;
        const long N = 1L << logn;
        const CrossConst ip = tab.cross[i * kMaxMods + np], il = tab.cross[i * kMaxMods + kl];
        const u64 xv = x[grp * xs + (long)i * N + j];
        const int c = grp & 1;
        const bool has_add = (add.mask >> c) & 1;
        const u64 av = has_add ? add.base[(grp >> 1) * add.sb + c * add.sc + (long)i * N + j] : 0;
        u64 *dst = out + ((long)grp * kl + i) * N + j;
        if (fp) {
            double val = fp_mul(u64_to_fp(xv) - __longlong_as_double((long long)v), ip.invd, p.qd, p.qinv);
            if (has_add) val += u64_to_fp(av);
            *dst = fp_to_u64(fp_mul(val, il.invd, p.qd, p.qinv), p.qd, p.qinv);
            return;
        }
        const u64 ext = red4(v, p.q, p.q2);
        u64 val = red2(shoup_lazy(sub_mod(xv, ext, p.q), ip.inv, ip.invs, p.q, p.qn), p.q);
        if (has_add) val = add_mod(val, av, p.q);
        *dst = red2(shoup_lazy(val, il.inv, il.invs, p.q, p.qn), p.q);
    }
    __device__ void store_inv(int, int, u64, const PrimeConst &) const {}
    __device__ void store_inv_fp(int, int, double, const PrimeConst &) const {}
};

// One workgroup per forward transform of an Op (load, transform, store_fwd). With xcd_order the
// `period` residues of a group (which read the same input words) run back to back on one XCD.
template <int LOGN, class Op>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_fwd_one(Op op, int count, int period, int xcd_order, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int T = Geo<LOGN>::T;
    const int tid = opaque(threadIdx.x);
    int r = blockIdx.x;
    if (xcd_order) {
        const int loc = blockIdx.x >> 3;
        r = ((loc / period) * 8 + (blockIdx.x & 7)) * period + loc % period;
    }
    if (r >= count) return;
    const int pi = op.prime(r);
    const PrimeConst p = tab.pc[pi];
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = op.load(r, tid + T * e, p, tab);
    const bool fp = fwd_transform<LOGN>(v, lds, tid, tab, pi, p);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int j = wave_elem(tid, e);
        op.store_fwd(r, j, lds[lds_idx(j)], fp, p, tab);
    }
}

// x[g][kl] += P a[g][kl] mod q_kl for the polynomials g = 2 b + c with an addend (see
// OpDropRescale). grid: x = N / 256, y = groups.
__global__ void __launch_bounds__(256)
k_fold_last(u64 *__restrict__ x, long xs, int kl, int np, DropAdd add, int logn, Tables tab) {
    const long N = 1L << logn;
    const int n = blockIdx.x * 256 + threadIdx.x, grp = blockIdx.y, c = grp & 1;
    if (!((add.mask >> c) & 1)) return;
    const PrimeConst p = tab.pc[kl];
    const u64 a = add.base[(grp >> 1) * add.sb + c * add.sc + (long)kl * N + n];
    u64 *xp = x + grp * xs + (long)kl * N + n;
    *xp = add_mod(*xp, mul_mod(a, tab.cross[kl * kMaxMods + np].qj_mod_qi, p), p.q);
}

template <int LOGN, class Op>
__global__ void __launch_bounds__(64)
k_fwd_top(Op op, u64 *__restrict__ tmp, int count, Tables tab) {
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, S = T / 64;
    const int r = blockIdx.x / S, tid = (blockIdx.x % S) * 64 + threadIdx.x;
    if (r >= count) return;
    if (op.copy_only(r)) {
#pragma unroll
        for (int e = 0; e < 16; ++e) op.copy(r, tid + T * e, tab);
        return;
    }
    const int pi = op.prime(r);
    const PrimeConst p = tab.pc[pi];
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = op.load(r, tid + T * e, p, tab);
    u64 *t = tmp + (long)r * N;
    if (p.fp) {
        double d[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = u64_to_fp(v[e]);
        fwd_pass_fp<LOGN, LOGN - 4, 4>(d, tid, reinterpret_cast<const double *>(tab.tws + (long)pi * N), p.qd, p.qinv);
#pragma unroll
        for (int e = 0; e < 16; ++e) t[tid + T * e] = (u64)__double_as_longlong(d[e]);
        return;
    }
    fwd_pass<LOGN, LOGN - 4, 4>(v, tid, tab.tw + (long)pi * N, tab.tws + (long)pi * N, p.q, p.q2, p.qn, p.nq2);
#pragma unroll
    for (int e = 0; e < 16; ++e) t[tid + T * e] = v[e];
}

template <int LOGN, class Op>
__global__ void __launch_bounds__(64)
k_fwd_sub(Op op, const u64 *__restrict__ tmp, int count, Tables tab) {
    __shared__ u64 lds[1024 + 32];
    constexpr int N = Geo<LOGN>::N, S = N / 1024;
    const int r = blockIdx.x / S, w = blockIdx.x % S, lane = threadIdx.x, tid = w * 64 + lane;
    if (r >= count || op.copy_only(r)) return;
    const int pi = op.prime(r);
    const PrimeConst p = tab.pc[pi];
    const u64 *t = tmp + (long)r * N + (w << 10);
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[lds_idx((e << 6) | lane)] = t[(e << 6) | lane];
    wave_sync();
    if (p.fp) {
        double d[16];
        const double *tw = reinterpret_cast<const double *>(tab.tws + (long)pi * N);
        fwd_sub_plan<LOGN>(d, reinterpret_cast<double *>(lds), lane, [&](auto lo, auto rb, auto wv) {
            fwd_pass_fp<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(d, tid, tw, p.qd, p.qinv);
        });
    } else {
        u64 v[16];
        const u64 *tw = tab.tw + (long)pi * N, *tws = tab.tws + (long)pi * N;
        fwd_sub_plan<LOGN>(v, lds, lane, [&](auto lo, auto rb, auto wv) {
            fwd_pass<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, tws, p.q, p.q2,
                                                                                        p.qn, p.nq2);
        });
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int jl = (e << 6) | lane;
        op.store_fwd(r, (w << 10) | jl, lds[lds_idx(jl)], p.fp != 0, p, tab);
    }
}

template <int LOGN, class Op>
__global__ void __launch_bounds__(64)
k_inv_sub(Op op, u64 *__restrict__ tmp, int count, Tables tab) {
    __shared__ u64 lds[1024 + 32];
    constexpr int N = Geo<LOGN>::N, S = N / 1024;
    const int r = blockIdx.x / S, w = blockIdx.x % S, lane = threadIdx.x, tid = w * 64 + lane;
    if (r >= count) return;
    const int pi = op.prime(r);
    const PrimeConst p = tab.pc[pi];
    u64 *t = tmp + (long)r * N + (w << 10);
    if (p.fp) {
        double *dl = reinterpret_cast<double *>(lds);
#pragma unroll
        for (int e = 0; e < 16; ++e) dl[lds_idx((e << 6) | lane)] = u64_to_fp(op.load(r, (w << 10) | (e << 6) | lane, p, tab));
        wave_sync();
        double d[16];
        const double *tw = reinterpret_cast<const double *>(tab.itws + (long)pi * N);
        inv_sub_plan<LOGN>(d, dl, lane, [&](auto lo, auto rb, auto wv) {
            inv_pass_fp<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(d, tid, tw, p.qd, p.qinv);
        });
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) lds[lds_idx((e << 6) | lane)] = op.load(r, (w << 10) | (e << 6) | lane, p, tab);
        wave_sync();
        u64 v[16];
        const u64 *tw = tab.itw + (long)pi * N, *tws = tab.itws + (long)pi * N;
        inv_sub_plan<LOGN>(v, lds, lane, [&](auto lo, auto rb, auto wv) {
            inv_pass<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, tws, p.q, p.q2,
                                                                                        p.qn, p.nq2);
        });
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) t[(e << 6) | lane] = lds[lds_idx((e << 6) | lane)];
}

template <int LOGN, class Op>
__global__ void __launch_bounds__(64)
k_inv_top(Op op, const u64 *__restrict__ tmp, int count, Tables tab) {
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, S = T / 64;
    const int r = blockIdx.x / S, tid = (blockIdx.x % S) * 64 + threadIdx.x;
    if (r >= count) return;
    const int pi = op.prime(r);
    const PrimeConst p = tab.pc[pi];
    const u64 *t = tmp + (long)r * N;
    if (p.fp) {
        double d[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = __longlong_as_double((long long)t[tid + T * e]);
        inv_pass_fp<LOGN, LOGN - 4, 4>(d, tid, reinterpret_cast<const double *>(tab.itws + (long)pi * N), p.qd, p.qinv);
#pragma unroll
        for (int e = 0; e < 16; ++e) op.store_inv_fp(r, tid + T * e, d[e], p);
        return;
    }
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = t[tid + T * e];
    inv_pass<LOGN, LOGN - 4, 4>(v, tid, tab.itw + (long)pi * N, tab.itws + (long)pi * N, p.q, p.q2, p.qn, p.nq2);
#pragma unroll
    for (int e = 0; e < 16; ++e) op.store_inv(r, tid + T * e, v[e], p);
}

template <class Op>
static void launch_split_fwd(int logn, const Op &op, u64 *tmp, int count, const Tables &tab, hipStream_t st) {
    const dim3 grid((unsigned)count << (logn - 10)), blk(64);
    switch (logn) {
        case 12:
            hipLaunchKernelGGL((k_fwd_top<12, Op>), grid, blk, 0, st, op, tmp, count, tab);
            hipLaunchKernelGGL((k_fwd_sub<12, Op>), grid, blk, 0, st, op, tmp, count, tab);
            break;
        case 13:
            hipLaunchKernelGGL((k_fwd_top<13, Op>), grid, blk, 0, st, op, tmp, count, tab);
            hipLaunchKernelGGL((k_fwd_sub<13, Op>), grid, blk, 0, st, op, tmp, count, tab);
            break;
        default:
            hipLaunchKernelGGL((k_fwd_top<14, Op>), grid, blk, 0, st, op, tmp, count, tab);
            hipLaunchKernelGGL((k_fwd_sub<14, Op>), grid, blk, 0, st, op, tmp, count, tab);
            break;
    }
}

template <class Op>
static void launch_split_inv(int logn, const Op &op, u64 *tmp, int count, const Tables &tab, hipStream_t st) {
    const dim3 grid((unsigned)count << (logn - 10)), blk(64);
    switch (logn) {
        case 12:
            hipLaunchKernelGGL((k_inv_sub<12, Op>), grid, blk, 0, st, op, tmp, count, tab);
            hipLaunchKernelGGL((k_inv_top<12, Op>), grid, blk, 0, st, op, tmp, count, tab);
            break;
        case 13:
            hipLaunchKernelGGL((k_inv_sub<13, Op>), grid, blk, 0, st, op, tmp, count, tab);
            hipLaunchKernelGGL((k_inv_top<13, Op>), grid, blk, 0, st, op, tmp, count, tab);
            break;
        default:
            hipLaunchKernelGGL((k_inv_sub<14, Op>), grid, blk, 0, st, op, tmp, count, tab);
            hipLaunchKernelGGL((k_inv_top<14, Op>), grid, blk, 0, st, op, tmp, count, tab);
            break;
    }
}

// Workgroup and dynamic LDS of the one-workgroup transforms.
static dim3 ntt_block(int logn) { return dim3(1u << (logn - 4)); }
static size_t ntt_lds(int logn) { return (size_t)((1 << logn) + ((1 << logn) >> 5)) * 8; }

// ---------------------------------------------------------------- looped transforms (many residues)
// With one residue per workgroup, the residue-sized LDS admits one workgroup per CU (at N = 2^14),
// which runs load -> passes -> store with the CU's memory traffic and its arithmetic in turn, and waits for
// the next workgroup's dispatch after its last wave ends. For launches of many residues, a grid of
// as many workgroups as fit on the CUs at once loops over the residues instead: while the waves transform one residue,
// the input lines of the next are brought into L2 (one word per line and thread, loop_touch), so
// that its loads at the next iteration are L2 hits; a second barrier per residue keeps the next
// exchange from overwriting LDS words that a slower wave still reads. Each arithmetic class (FP64 or integer
// primes) is a kernel of its own, launched over the residues of its primes, so that each is held
// to its own register budget. Every butterfly is the one of the one-workgroup form, so the
// residues are the same. The lift and the combine come from the Op (fetch / prep / store_*).
//
// The residues of a launch are numbered in periods (the k + 1 targets of a ModUp digit, the k
// primes of a ModDown group); those of the kernel's class are the r with r mod period in pos.
// Period d goes to XCD d mod 8 (workgroup b runs on XCD b mod 8), and the S workgroups of an XCD
// take its residues in turn, so the residues of one period, which read the same input words, run
// at the same time on one L2.

struct SlotSet {
    int period, n;
    int pos[kMaxMods];
};

struct LoopUnits {
    int x, S, U, count;
};
__device__ __forceinline__ LoopUnits loop_units(const SlotSet &ss, int count) {
    LoopUnits lu;
    lu.x = blockIdx.x & 7;
    lu.S = gridDim.x >> 3;
    lu.count = count;
    const int D = (count + ss.period - 1) / ss.period;
    lu.U = (D > lu.x ? (D - 1 - lu.x) / 8 + 1 : 0) * ss.n;
    return lu;
}
__device__ __forceinline__ int loop_residue(const LoopUnits &lu, const SlotSet &ss, int u) {
    return ((u / ss.n) * 8 + lu.x) * ss.period + ss.pos[u % ss.n];
}
__device__ __forceinline__ int loop_next(const LoopUnits &lu, const SlotSet &ss, int u) {
    for (u += lu.S; u < lu.U && loop_residue(lu, ss, u) >= lu.count; u += lu.S) {}
    return u;
}
__device__ __forceinline__ int loop_first(const LoopUnits &lu, const SlotSet &ss) {
    const int u = blockIdx.x >> 3;
    return u < lu.U && loop_residue(lu, ss, u) >= lu.count ? loop_next(lu, ss, u) : u;
}

// Bring the input lines of residue u into L2: each thread loads one word of its own 128-byte line
// (16 T words = one residue). The loaded word is kept until the end of the iteration (keep), so
// the load is neither dropped nor waited for before then.
template <int LOGN, class Op>
__device__ __forceinline__ u64 loop_touch(const Op &op, const LoopUnits &lu, const SlotSet &ss, int u) {
    if (u >= lu.U) return 0;
    const int r = loop_residue(lu, ss, u);
    if (op.copy_only(r)) return 0;
    return op.fetch(r, opaque(threadIdx.x) * 16);
}
__device__ __forceinline__ void keep(u64 x) { asm volatile("" ::"v"(x)); }

template <int LOGN, class Op, bool FP>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_fwd_loop(Op op, SlotSet ss, int count, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, TOP = LOGN - 4;
    const LoopUnits lu = loop_units(ss, count);
    for (int u = loop_first(lu, ss); u < lu.U;) {
        const int r = loop_residue(lu, ss, u), un = loop_next(lu, ss, u);
        const int pi = op.prime(r);
        const PrimeConst p = tab.pc[pi];
        const int tid = opaque(threadIdx.x);
        if (op.copy_only(r)) {
            const u64 t = loop_touch<LOGN>(op, lu, ss, un);
#pragma unroll
            for (int e = 0; e < 16; ++e) op.copy(r, tid + T * e, tab);
            keep(t);
            u = un;
            continue;
        }
        if constexpr (FP) {
            double d[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) d[e] = u64_to_fp(op.load(r, tid + T * e, p, tab));
            const u64 t = loop_touch<LOGN>(op, lu, ss, un);
            const double *tw = reinterpret_cast<const double *>(tab.tws + (long)pi * N);
            double *dl = reinterpret_cast<double *>(lds);
            fwd_pass_fp<LOGN, TOP, 4>(d, tid, tw, p.qd, p.qinv);
            __syncthreads();                      // every wave is done with the previous residue's LDS
            to_lds<LOGN, TOP, 4>(d, dl, tid);
            __syncthreads();
            fwd_sub_plan<LOGN>(d, dl, tid, [&](auto lo, auto rb, auto wv) {
                fwd_pass_fp<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(d, tid, tw, p.qd,
                                                                                               p.qinv);
            });
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int j = wave_elem(tid, e);
                op.store_fwd(r, j, lds[lds_idx(j)], true, p, tab);
            }
            keep(t);
        } else {
            u64 v[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = op.load(r, tid + T * e, p, tab);
            const u64 t = loop_touch<LOGN>(op, lu, ss, un);
            const u64 *tw = tab.tw + (long)pi * N, *tws = tab.tws + (long)pi * N;
            fwd_pass<LOGN, TOP, 4>(v, tid, tw, tws, p.q, p.q2, p.qn, p.nq2);
            __syncthreads();
            to_lds<LOGN, TOP, 4>(v, lds, tid);
            __syncthreads();
            fwd_sub_plan<LOGN>(v, lds, tid, [&](auto lo, auto rb, auto wv) {
                fwd_pass<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, tws, p.q,
                                                                                            p.q2, p.qn, p.nq2);
            });
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int j = wave_elem(tid, e);
                op.store_fwd(r, j, lds[lds_idx(j)], false, p, tab);
            }
            keep(t);
        }
        u = un;
    }
}

template <int LOGN, class Op, bool FP>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_inv_loop(Op op, SlotSet ss, int count, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, TOP = LOGN - 4;
    const LoopUnits lu = loop_units(ss, count);
    for (int u = loop_first(lu, ss); u < lu.U;) {
        const int r = loop_residue(lu, ss, u), un = loop_next(lu, ss, u);
        const int pi = op.prime(r);
        const PrimeConst p = tab.pc[pi];
        const int tid = opaque(threadIdx.x);
        u64 x[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = op.load(r, wave_elem(tid, e), p, tab);
        const u64 t = loop_touch<LOGN>(op, lu, ss, un);
        __syncthreads();                          // every wave is done with the previous residue's LDS
        if constexpr (FP) {
            double *dl = reinterpret_cast<double *>(lds);
#pragma unroll
            for (int e = 0; e < 16; ++e) dl[lds_idx(wave_elem(tid, e))] = u64_to_fp(x[e]);
            wave_sync();
            double d[16];
            const double *tw = reinterpret_cast<const double *>(tab.itws + (long)pi * N);
            inv_sub_plan<LOGN>(d, dl, tid, [&](auto lo, auto rb, auto wv) {
                inv_pass_fp<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(d, tid, tw, p.qd,
                                                                                               p.qinv);
            });
            __syncthreads();
            from_lds<LOGN, TOP, 4>(d, dl, tid);
            inv_pass_fp<LOGN, TOP, 4>(d, tid, tw, p.qd, p.qinv);
#pragma unroll
            for (int e = 0; e < 16; ++e) op.store_inv_fp(r, tid + T * e, d[e], p);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) lds[lds_idx(wave_elem(tid, e))] = x[e];
            wave_sync();
            u64 v[16];
            const u64 *tw = tab.itw + (long)pi * N, *tws = tab.itws + (long)pi * N;
            inv_sub_plan<LOGN>(v, lds, tid, [&](auto lo, auto rb, auto wv) {
                inv_pass<LOGN, decltype(lo)::value, decltype(rb)::value, decltype(wv)::value>(v, tid, tw, tws, p.q,
                                                                                            p.q2, p.qn, p.nq2);
            });
            __syncthreads();
            from_lds<LOGN, TOP, 4>(v, lds, tid);
            inv_pass<LOGN, TOP, 4>(v, tid, tw, tws, p.q, p.q2, p.qn, p.nq2);
#pragma unroll
            for (int e = 0; e < 16; ++e) op.store_inv(r, tid + T * e, v[e], p);
        }
        keep(t);
        u = un;
    }
}

// The slots of a period of residue primes `prime[0..period)` by class (0: FP64, 1: integer).
static void class_slots(const int *prime, int period, const Tables &tab, SlotSet (&ss)[2]) {
    ss[0] = SlotSet{period, 0, {}};
    ss[1] = SlotSet{period, 0, {}};
    for (int i = 0; i < period; ++i) {
        SlotSet &s = ss[tab.host_fp[prime[i]] ? 0 : 1];
        s.pos[s.n++] = i;
    }
}

template <int LOGN, bool INV, class Op>
static void launch_loop_one(const Op &op, const SlotSet (&ss)[2], int count, const Tables &tab, hipStream_t st,
                            int cls) {
    const size_t sh = ntt_lds(LOGN);
    const int per_cu = (size_t)tab.lds_cu >= 2 * sh ? (int)((size_t)tab.lds_cu / sh) : 1;   // resident per CU
    const dim3 grid((unsigned)((tab.cus & ~7) * per_cu)), blk = ntt_block(LOGN);
    for (int c = 0; c < 2; ++c) {
        if (ss[c].n == 0 || (cls >= 0 && c != cls)) continue;
        if constexpr (INV) {
            if (c == 0) hipLaunchKernelGGL((k_inv_loop<LOGN, Op, true>), grid, blk, sh, st, op, ss[c], count, tab);
            else hipLaunchKernelGGL((k_inv_loop<LOGN, Op, false>), grid, blk, sh, st, op, ss[c], count, tab);
        } else {
            if (c == 0) hipLaunchKernelGGL((k_fwd_loop<LOGN, Op, true>), grid, blk, sh, st, op, ss[c], count, tab);
            else hipLaunchKernelGGL((k_fwd_loop<LOGN, Op, false>), grid, blk, sh, st, op, ss[c], count, tab);
        }
    }
}

template <bool INV, class Op>
static void launch_loop(int logn, const Op &op, const int *prime, int period, int count, const Tables &tab,
                        hipStream_t st, int cls) {
    SlotSet ss[2];
    class_slots(prime, period, tab, ss);
    switch (logn) {
        case 12: launch_loop_one<12, INV>(op, ss, count, tab, st, cls); break;
        case 13: launch_loop_one<13, INV>(op, ss, count, tab, st, cls); break;
        default: launch_loop_one<14, INV>(op, ss, count, tab, st, cls); break;
    }
}

// A launch loops when each arithmetic class among its residues has at least kn.ntt_loop residues
// per CU (0: never): each class is a launch of its own with a fixed share of residues per
// workgroup, and few residues per CU would leave a tail of idle CUs behind each.
static int loop_mask(int count, const int *prime, int period, const Tables &tab, const Knobs &kn) {
    if (kn.ntt_loop <= 0 || tab.cus < 8 || period <= 0) return 0;
    long per_class[2] = {0, 0};
    for (int i = 0; i < period; ++i) {
        const long n = count / period + (i < count % period ? 1 : 0);
        per_class[tab.host_fp[prime[i]] ? 0 : 1] += n;
    }
    int mask = 0;
    for (int c = 0; c < 2; ++c) {
        if (per_class[c] > 0 && per_class[c] < (long)kn.ntt_loop * tab.cus) return 0;
        if (per_class[c] > 0) mask |= 1 << c;
    }
    return mask;
}
static bool use_loop(int count, const int *prime, int period, const Tables &tab, const Knobs &kn) {
    return loop_mask(count, prime, period, tab, kn) != 0;
}

static void modup_primes(int k, int nq, int (&prime)[kMaxMods]) {
    for (int t = 0; t <= k; ++t) prime[t] = t < k ? t : nq;
}
static void drop_primes(int k, int (&prime)[kMaxMods]) {
    for (int i = 0; i < k; ++i) prime[i] = i;
}

int ntt_loop_classes(int count, const ResMap &imap, const Tables &tab, const Knobs &kn, const u64 *split_tmp) {
    return split_tmp || count <= 0 ? 0 : loop_mask(count, imap.prime, imap.per, tab, kn);
}
int modup_loop_classes(int groups, int k, int nq, const Tables &tab, const Knobs &kn, const u64 *split_tmp) {
    if (split_tmp || groups <= 0) return 0;
    int prime[kMaxMods];
    modup_primes(k, nq, prime);
    return loop_mask(groups * k * (k + 1), prime, k + 1, tab, kn);
}
int drop_loop_classes(int groups, int k, const Tables &tab, const Knobs &kn, const u64 *split_tmp) {
    if (split_tmp || groups <= 0) return 0;
    int prime[kMaxMods];
    drop_primes(k, prime);
    return loop_mask(groups * k, prime, k, tab, kn);
}

// ---------------------------------------------------------------- split chains (few residues)
// ModUp, ModDown and rescale each run an inverse transform whose coefficients only feed the lifts
// of the forward transforms after it (a ModUp digit to its k + 1 targets, the dropped prime to the
// other k). In split form the chain is k_inv_sub over the inverse's residues, one kernel in which
// workgroup (r, t, s) runs the inverse's top pass of residue r (the one-workgroup form's inverse
// result, scaled by N^{-1}) and then, on the same 16 coefficients per thread, the lift and the
// forward top pass of target t of r, and k_fwd_sub over the targets: three launches instead of four,
// and the coefficients never leave registers. The inverse's top pass is recomputed per target, on
// CUs that a launch of a few residues leaves idle anyway. Target u = r per + t of the forward Op.
// The inverse's top pass of one residue of prime pi whose wave-local passes k_inv_sub left in ti,
// scaled by N^-1: canonical coefficients tid + T e.
template <int LOGN>
__device__ __forceinline__ void inv_top_coeffs(const u64 *__restrict__ ti, int pi, int tid, const Tables &tab,
                                               u64 (&cf)[16]) {
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, TOP = LOGN - 4;
    const PrimeConst p = tab.pc[pi];
    if (p.fp) {
        double d[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = __longlong_as_double((long long)ti[tid + T * e]);
        inv_pass_fp<LOGN, TOP, 4>(d, tid, reinterpret_cast<const double *>(tab.itws + (long)pi * N), p.qd, p.qinv);
#pragma unroll
        for (int e = 0; e < 16; ++e) cf[e] = fp_to_u64(fp_mul(d[e], p.ninvd, p.qd, p.qinv), p.qd, p.qinv);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) cf[e] = ti[tid + T * e];
        inv_pass<LOGN, TOP, 4>(cf, tid, tab.itw + (long)pi * N, tab.itws + (long)pi * N, p.q, p.q2, p.qn, p.nq2);
#pragma unroll
        for (int e = 0; e < 16; ++e) cf[e] = red2(shoup_lazy(cf[e], p.ninv, p.ninvs, p.q, p.qn), p.q);
    }
}

template <int LOGN, class OpF>
__global__ void __launch_bounds__(64)
k_inv_fwd_top(OpNtt opi, OpF opf, const u64 *__restrict__ tmp_i, u64 *__restrict__ tmp_f, int count_i, int per,
              Tables tab) {
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, S = T / 64, TOP = LOGN - 4;
    const int ri = blockIdx.x / (S * per), t = (blockIdx.x / S) % per, tid = (blockIdx.x % S) * 64 + threadIdx.x;
    if (ri >= count_i) return;
    const int rf = ri * per + t;
    if (opf.copy_only(rf)) {
#pragma unroll
        for (int e = 0; e < 16; ++e) opf.copy(rf, tid + T * e, tab);
        return;
    }
    u64 cf[16];                                   // canonical coefficients of residue ri
    inv_top_coeffs<LOGN>(tmp_i + (long)ri * N, opi.prime(ri), tid, tab, cf);
    const int pf = opf.prime(rf);
    const PrimeConst q = tab.pc[pf];
    u64 *tf = tmp_f + (long)rf * N;
    if (q.fp) {
        double d[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = u64_to_fp(opf.prep(rf, cf[e], q, tab));
        fwd_pass_fp<LOGN, TOP, 4>(d, tid, reinterpret_cast<const double *>(tab.tws + (long)pf * N), q.qd, q.qinv);
#pragma unroll
        for (int e = 0; e < 16; ++e) tf[tid + T * e] = (u64)__double_as_longlong(d[e]);
        return;
    }
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = opf.prep(rf, cf[e], q, tab);
    fwd_pass<LOGN, TOP, 4>(v, tid, tab.tw + (long)pf * N, tab.tws + (long)pf * N, q.q, q.q2, q.qn, q.nq2);
#pragma unroll
    for (int e = 0; e < 16; ++e) tf[tid + T * e] = v[e];
}

template <int LOGN, class OpF>
static void launch_chain_one(bool inverse_part, const OpNtt &opi, int count_i, const OpF &opf, int per, u64 *tmp_i,
                             u64 *tmp_f, const Tables &tab, hipStream_t st) {
    const dim3 blk(64);
    if (inverse_part) {
        hipLaunchKernelGGL((k_inv_sub<LOGN, OpNtt>), dim3((unsigned)count_i << (LOGN - 10)), blk, 0, st, opi, tmp_i,
                           count_i, tab);
        return;
    }
    const int count_f = count_i * per;
    hipLaunchKernelGGL((k_inv_fwd_top<LOGN, OpF>), dim3((unsigned)count_f << (LOGN - 10)), blk, 0, st, opi, opf, tmp_i,
                       tmp_f, count_i, per, tab);
    hipLaunchKernelGGL((k_fwd_sub<LOGN, OpF>), dim3((unsigned)count_f << (LOGN - 10)), blk, 0, st, opf, tmp_f, count_f,
                       tab);
}

// Split chain of the one-pass ModDown and rescale (OpDropRescale): k_inv_sub over the two
// coefficient rows of each polynomial g (residues 2 g: row kl, 2 g + 1: the P row), then workgroup
// (g, t, s) runs the inverse's top pass of both rows on its 16 coefficients per thread, forms the
// lift of target t from them (OpDropRescale::combine) and runs its forward top pass; k_fwd_sub
// over the g kl + t targets finishes.
template <int LOGN>
__global__ void __launch_bounds__(64)
k_inv2_fwd_top(OpDropRescale opf, const u64 *__restrict__ tmp_i, u64 *__restrict__ tmp_f, int groups, Tables tab) {
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T, S = T / 64, TOP = LOGN - 4;
    const int kl = opf.kl;
    const int g = blockIdx.x / (S * kl), t = (blockIdx.x / S) % kl, tid = (blockIdx.x % S) * 64 + threadIdx.x;
    if (g >= groups) return;
    const int rf = g * kl + t;
    u64 cl[16], cp[16];
    inv_top_coeffs<LOGN>(tmp_i + (long)(2 * g) * N, kl, tid, tab, cl);
    inv_top_coeffs<LOGN>(tmp_i + (long)(2 * g + 1) * N, opf.np, tid, tab, cp);
    const PrimeConst q = tab.pc[t];
    u64 *tf = tmp_f + (long)rf * N;
    if (q.fp) {
        double d[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) d[e] = u64_to_fp(opf.combine(rf, cl[e], cp[e], q, tab));
        fwd_pass_fp<LOGN, TOP, 4>(d, tid, reinterpret_cast<const double *>(tab.tws + (long)t * N), q.qd, q.qinv);
#pragma unroll
        for (int e = 0; e < 16; ++e) tf[tid + T * e] = (u64)__double_as_longlong(d[e]);
        return;
    }
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = opf.combine(rf, cl[e], cp[e], q, tab);
    fwd_pass<LOGN, TOP, 4>(v, tid, tab.tw + (long)t * N, tab.tws + (long)t * N, q.q, q.q2, q.qn, q.nq2);
#pragma unroll
    for (int e = 0; e < 16; ++e) tf[tid + T * e] = v[e];
}

template <int LOGN>
static void launch_drop_rescale_chain_one(bool inverse_part, const OpNtt &opi, const OpDropRescale &opf, int groups,
                                          u64 *tmp_i, u64 *tmp_f, const Tables &tab, hipStream_t st) {
    const dim3 blk(64);
    if (inverse_part) {
        hipLaunchKernelGGL((k_inv_sub<LOGN, OpNtt>), dim3((unsigned)(2 * groups) << (LOGN - 10)), blk, 0, st, opi, tmp_i,
                           2 * groups, tab);
        return;
    }
    const int count_f = groups * opf.kl;
    hipLaunchKernelGGL(k_inv2_fwd_top<LOGN>, dim3((unsigned)count_f << (LOGN - 10)), blk, 0, st, opf, tmp_i, tmp_f,
                       groups, tab);
    hipLaunchKernelGGL((k_fwd_sub<LOGN, OpDropRescale>), dim3((unsigned)count_f << (LOGN - 10)), blk, 0, st, opf,
                       tmp_f, count_f, tab);
}

template <class OpF>
static void launch_chain(int logn, bool inverse_part, const OpNtt &opi, int count_i, const OpF &opf, int per,
                         u64 *tmp_i, u64 *tmp_f, const Tables &tab, hipStream_t st) {
    switch (logn) {
        case 12: launch_chain_one<12>(inverse_part, opi, count_i, opf, per, tmp_i, tmp_f, tab, st); break;
        case 13: launch_chain_one<13>(inverse_part, opi, count_i, opf, per, tmp_i, tmp_f, tab, st); break;
        default: launch_chain_one<14>(inverse_part, opi, count_i, opf, per, tmp_i, tmp_f, tab, st); break;
    }
}

void launch_modup_chain(int logn, bool inverse_part, const u64 *d, const ResMap &dmap, u64 *digits, int groups, int k,
                        int nq, const Tables &tab, hipStream_t st, u64 *tmp_i, u64 *tmp_f) {
    if (groups <= 0) return;
    const OpNtt opi{d, dmap, nullptr, ResMap{}, logn};
    launch_chain(logn, inverse_part, opi, groups * k, OpModup{nullptr, d, dmap, digits, k, nq, logn}, k + 1, tmp_i,
                 tmp_f, tab, st);
}

void launch_drop_chain(int logn, bool inverse_part, const u64 *in, const ResMap &imap, const u64 *x, const GrpMap &xm,
                       u64 *out, int groups, int k, int drop, const DropAdd &add, const Tables &tab, hipStream_t st,
                       u64 *tmp_i, u64 *tmp_f) {
    if (groups <= 0) return;
    const OpNtt opi{in, imap, nullptr, ResMap{}, logn};
    launch_chain(logn, inverse_part, opi, groups, OpDrop{x, xm, nullptr, out, k, drop, logn, add}, k, tmp_i, tmp_f,
                 tab, st);
}

// Signed 64-bit coefficients -> residues mod q_p -> NTT. src: dense [G][N] int64; out: [G][P][N]
// for the P prime indices plist[0..P).
template <int LOGN>
__global__ void __launch_bounds__(Geo<LOGN>::T)
k_int_ntt(const int64_t *__restrict__ src, u64 *__restrict__ out, PrimeList pl, Tables tab) {
    extern __shared__ u64 lds[];
    constexpr int N = Geo<LOGN>::N, T = Geo<LOGN>::T;
    const int tid = opaque(threadIdx.x);
    const int slot = blockIdx.x % pl.n, grp = blockIdx.x / pl.n;
    const int pi = pl.idx[slot];
    const PrimeConst p = tab.pc[pi];
    const int64_t *s = src + (long)grp * N;
    u64 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int64_t a = s[tid + T * e];
        const u64 m = reduce_any((u64)(a < 0 ? -a : a), p);
        v[e] = a < 0 ? neg_mod(m, p.q) : m;
    }
    const bool fp = fwd_transform<LOGN>(v, lds, tid, tab, pi, p);
    u64 *dst = out + ((long)grp * pl.n + slot) * N;
#pragma unroll
    for (int e = 0; e < 16; ++e) dst[wave_elem(tid, e)] = fwd_result(lds, wave_elem(tid, e), fp, p);
}

// ---------------------------------------------------------------- 30-bit limb products
// For a prime below 2^60 every residue splits as x = xh 2^30 + xl with xh, xl < 2^30, and a
// product x w is four 30 x 30-bit products (each below 2^60) that v_mad_u64_u32 adds into 64-bit
// column sums of weights 1, 2^30 and 2^60 without carries; a column takes 16 such products
// before it could reach 2^64. The value is reduced mod q once, from its 128-bit form.
constexpr u64 kM30 = (1ull << 30) - 1;

// c2 only has to come back below 2^63 here (8 more terms then add < 2^63 + 2^34). When 2^60 mod q
// is below 2^58 (primes near 2^60), c2 = t 2^60 + u with t < 16 is replaced by the congruent
// t (2^60 mod q) + u < 2^60 + 15 2^58 < 2^62; for other primes it is reduced mod q.
__device__ __forceinline__ void limb_normalize(u64 (&c)[3], const PrimeConst &p) {
    c[1] += c[0] >> 30;
    c[0] &= kM30;
    c[2] += c[1] >> 30;
    c[1] &= kM30;
    if (p.r60 < (1ull << 58)) c[2] = (c[2] & ((1ull << 60) - 1)) + (u64)(u32)(c[2] >> 60) * p.r60;
    else c[2] = reduce_any(c[2], p);
}

// L + h 2^60 mod q for L < 2^60, any h < 2^64 and q < 2^60: h 2^60 is congruent to h (2^60 mod q),
// a Shoup product in [0, 2q); the sum is below 4q when q >= 2^59 (two conditional subtracts) and
// below 2^62 otherwise (one general reduction).
__device__ __forceinline__ u64 limb_fold60(u64 l, u64 h, const PrimeConst &p) {
    const u64 s = l + shoup_lazy(h, p.r60, p.r60s, p.q, p.qn);
    return (p.q >> 59) ? red4(s, p.q, p.q2) : reduce_any(s, p);
}
// c0 + c1 2^30 + c2 2^60 = L + c2 2^60 with L < 2^60 once normalized.
__device__ __forceinline__ u64 limb_reduce(u64 (&c)[3], const PrimeConst &p) {
    limb_normalize(c, p);
    return limb_fold60(c[0] | (c[1] << 30), c[2], p);
}

// (c0 + (c1 + c2) 2^30 + c3 2^60) mod q for q below 2^60, each column below 2^64 - 2^61: the
// weight-2^30 columns are carried so that the value is L + h 2^60 with L < 2^60 and
// h < c3 + 2^35.
__device__ __forceinline__ u64 limb_reduce4(const u64 (&c)[4], const PrimeConst &p) {
    const u64 u = (c[0] >> 30) + (c[1] & kM30) + (c[2] & kM30);     // below 2^35
    const u64 l = (c[0] & kM30) | ((u & kM30) << 30);
    const u64 h = c[3] + (c[1] >> 30) + (c[2] >> 30) + (u >> 30);
    return limb_fold60(l, h, p);
}

// ---------------------------------------------------------------- elementwise kernels
// Key inner product with the automorphism fused into the digit gather:
//   out[b][r][0][t] = sum_j D[b][r][j][t][sigma_r] * key_r[j][0][t] (+ fold),  out[..][1][t]
//   likewise with key_r[j][1][t]; t = 0..k (k = the special prime). D: digits + b db + r dr +
//   (j (k+1) + t) N, as ModUp stores them (FP64 bit patterns for FP64 primes);
//   out[b][r] at out + b ob + r 2 (k+1) N. For rows t < fold.rows, polynomial 0
//   also gets fold.mul[t] * fold.src[b sb + r sr + t N] gathered through sigma_r (the P sigma(c0)
//   term of a baby step kept over Q*P, or the sigma(c0) of a giant step's extended operand).
// One workgroup per (source tile of 256 coefficients, t, group of RR rotations); each thread
// loops over the batch so a key word is read from HBM once per launch. A thread reads the digits
// (and the fold term) at its source coefficient m once and, for each rotation r of its group,
// writes output coefficient n = sigma_r^{-1}(m), so that the digit loads are contiguous; in
// bit-reversed evaluation order the automorphism permutes aligned blocks of 2^j coefficients
// among themselves, so n stays inside one aligned 256-block and the key loads and output stores
// of a wave stay within 512 bytes. Hoisted rotations all read the same digit words: RR of them per
// workgroup divide the digit reads (served by L2, and the key product's limit at RR = 1) by RR.
// Workgroups are dealt to the 8 XCDs in turn (id mod 8); with xcd set the 1D grid is numbered
// such that all rotation groups of one (source tile, t) run back to back on the same XCD (with
// hoisted digits, dr = 0, they read the same digit words, which its L2 serves); otherwise tiles
// vary fastest, then t, then the rotation group.
//
// The rows of one launch (RowSet) all take one arithmetic class (KeyipClass), and each class is
// its own kernel, so that each gets the register budget of its own products: k_keyip_fp (FP64
// primes), k_keyip_limb (30-bit limbs, primes below 2^60) and k_keyip (128-bit sums).
template <int K, int RR, int CLS>
__device__ __forceinline__ void
keyip_body(const u64 *__restrict__ digits, long db, long dr, const KeyList &keys, u64 *__restrict__ out, long ob,
           const KeyFold &fold, const RowSet &rows, int B, int R, int nq, int logn, int xcd_order,
           const PrimeConst *__restrict__ pcs) {
    const int nt = rows.n;
    const int pairs = nt << (logn - 8);
    const int RG = (R + RR - 1) / RR;                       // groups of RR rotations
    int rg, pair;
    if (xcd_order) {
        const int id = blockIdx.x, xcd = id & 7, j = id >> 3;
        rg = j % RG;
        pair = (j / RG) * 8 + xcd;                           // pair = tile * nt + row
    } else {
        const int tiles = 1 << (logn - 8), id = blockIdx.x;
        rg = id / pairs;
        pair = (id % tiles) * nt + (id / tiles) % nt;
    }
    if (pair >= pairs || rg >= RG) return;
    const int m = (pair / nt) * 256 + threadIdx.x;          // source coefficient
    const int t = rows.t[pair % nt];
    const int N = 1 << logn, np = nq + 1;
    const int pt = t < K ? t : nq;
    const PrimeConst p = pcs[pt];
    const int r0 = rg * RR, nr = R - r0 < RR ? R - r0 : RR;  // rotations r0 .. r0 + nr - 1
    const int src = m;
    const bool fd = fold.src != nullptr && t < fold.rows;            // uniform per workgroup
    const u64 fm = fd ? fold.mul[t] : 0;
    // Rotation rr of the group: its key, the output that gathers from m, its output offset. A
    // group short of RR rotations repeats its last one and drops that one's stores.
    const u64 *key[RR];
    int voff_o[RR];
    bool live[RR];
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
        const int r = r0 + (rr < nr ? rr : nr - 1);
        live[rr] = rr < nr;
        key[rr] = keys.key[r];
        const int n = keys.gal[r] == 1 ? m : galois_src(m, keys.ginv[r], logn);
        voff_o[rr] = (int)(((long)r * 2 * (K + 1) * N + (long)t * N + n) * 8);
    }
    // Batch loop. Ciphertext b's K digit words (and its fold word) come from buffer loads whose
    // address is a per-lane offset plus scalar parts (no per-load address arithmetic on the
    // VALU), one ciphertext ahead of the products; ciphertexts go in pairs so that the prefetched
    // words need no copies. With RR > 1 the rotations of the group share the digit words (the
    // launcher uses it only for hoisted digits, dr = 0, and a fold shared by the rotations).
    const int voff_d = (int)(((long)t * N + src) * 8);
    const int voff_f = fd ? (int)(((long)r0 * fold.sr + (long)t * N + src) * 8) : 0;
    const int rec_d = K * (K + 1) * N * 8, rec_o = (int)(ob * 8), rec_f = fd ? (int)(fold.sb * 8) : 0;
    const int sd = (K + 1) * N * 8;                                    // digit j at + j sd bytes
    const u64 *dbase = digits + r0 * dr;
    auto load = [&](int b, u64 (&x)[K], u64 &f, bool fold_on) {
        const BufRsrc rd = buf_rsrc(dbase + b * db, rec_d);
#pragma unroll
        for (int j = 0; j < K; ++j) x[j] = buf_load(rd, voff_d, j * sd);
        if (fold_on) f = buf_load(buf_rsrc(fold.src + b * fold.sb, rec_f), voff_f, 0);
    };
    auto store = [&](int b, int rr, u64 v0, u64 v1) {
        const BufRsrc ro = buf_rsrc(out + b * ob, live[rr] ? rec_o : 0);   // 0 bytes: stores dropped
        buf_store(v0, ro, voff_o[rr], 0);
        buf_store(v1, ro, voff_o[rr], sd);
    };
    // pairs (b, b + 1): xa holds b, xb is filled with b + 1 while b is multiplied, then xa with b + 2
    auto batch = [&](auto fold_tag, auto &&product) {
        constexpr bool FOLD = decltype(fold_tag)::value;
        u64 xa[K], xb[K], fa = 0, fb = 0;
        load(0, xa, fa, FOLD);
        for (int b = 0; b < B; b += 2) {
            const bool two = b + 1 < B;
            if (two) load(b + 1, xb, fb, FOLD);
            product(b, xa, fa);
            if (two) {
                if (b + 2 < B) load(b + 2, xa, fa, FOLD);
                product(b + 1, xb, fb);
            }
        }
    };
    // each key word is read once per launch (held in registers over the batch loop), so its loads
    // are non-temporal and leave L2 to the digit words that the rotations of a tile share
    if constexpr (CLS == KIP_FP) {
        // FP64 products (prime < 2^41): each term |.| <= 0.52 q, sums stay far below 2^53
        double kb[RR][K], ka[RR][K];
#pragma unroll
        for (int rr = 0; rr < RR; ++rr)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = (voff_o[rr] >> 3) % N;
                kb[rr][j] = u64_to_fp(__builtin_nontemporal_load(&key[rr][((long)(j * 2 + 0) * np + pt) * N + n]));
                ka[rr][j] = u64_to_fp(__builtin_nontemporal_load(&key[rr][((long)(j * 2 + 1) * np + pt) * N + n]));
            }
        const double fmd = u64_to_fp(fm);
        auto run = [&](auto fold_tag) {
            constexpr bool FOLD = decltype(fold_tag)::value;
            batch(fold_tag, [&](int b, const u64 (&x)[K], u64 fx) {
                double xd[K];
#pragma unroll
                for (int j = 0; j < K; ++j) xd[j] = __longlong_as_double((long long)x[j]);   // FP64 digit (ModUp)
                const double f = FOLD ? fp_mul(u64_to_fp(fx), fmd, p.qd, p.qinv) : 0.0;
#pragma unroll
                for (int rr = 0; rr < RR; ++rr) {
                    double a0 = f, a1 = 0.0;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        a0 += fp_mul(xd[j], kb[rr][j], p.qd, p.qinv);
                        a1 += fp_mul(xd[j], ka[rr][j], p.qd, p.qinv);
                    }
                    store(b, rr, fp_to_u64(a0, p.qd, p.qinv), fp_to_u64(a1, p.qd, p.qinv));
                }
            });
        };
        if (fd) run(std::true_type{});
        else run(std::false_type{});
    } else if constexpr (CLS == KIP_LIMB) {
        // prime below 2^60: 30-bit limb products into carry-free column sums (see k_mac_limb);
        // with the two cross products in separate columns every column takes 16 terms, and a
        // sum has at most K + 1 <= 9
        u32 bl[RR][K], bh[RR][K], al[RR][K], ah[RR][K];
#pragma unroll
        for (int rr = 0; rr < RR; ++rr)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = (voff_o[rr] >> 3) % N;
                const u64 b0 = key[rr][((long)(j * 2 + 0) * np + pt) * N + n];
                const u64 a0 = key[rr][((long)(j * 2 + 1) * np + pt) * N + n];
                bl[rr][j] = (u32)b0 & (u32)kM30;
                bh[rr][j] = (u32)(b0 >> 30);
                al[rr][j] = (u32)a0 & (u32)kM30;
                ah[rr][j] = (u32)(a0 >> 30);
            }
        const u32 fml = (u32)fm & (u32)kM30, fmh = (u32)(fm >> 30);
        auto run = [&](auto fold_tag) {
            constexpr bool FOLD = decltype(fold_tag)::value;
            batch(fold_tag, [&](int b, const u64 (&x)[K], u64 fx) {
                u32 xl[K], xh[K];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    xl[j] = (u32)x[j] & (u32)kM30;
                    xh[j] = (u32)(x[j] >> 30);
                }
#pragma unroll
                for (int rr = 0; rr < RR; ++rr) {
                    u64 c0[4] = {0, 0, 0, 0}, c1[4] = {0, 0, 0, 0};
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        c0[0] += (u64)xl[j] * bl[rr][j];
                        c0[1] += (u64)xl[j] * bh[rr][j];
                        c0[2] += (u64)xh[j] * bl[rr][j];
                        c0[3] += (u64)xh[j] * bh[rr][j];
                        c1[0] += (u64)xl[j] * al[rr][j];
                        c1[1] += (u64)xl[j] * ah[rr][j];
                        c1[2] += (u64)xh[j] * al[rr][j];
                        c1[3] += (u64)xh[j] * ah[rr][j];
                    }
                    if constexpr (FOLD) {
                        const u32 fl = (u32)fx & (u32)kM30, fh = (u32)(fx >> 30);
                        c0[0] += (u64)fl * fml;
                        c0[1] += (u64)fl * fmh;
                        c0[2] += (u64)fh * fml;
                        c0[3] += (u64)fh * fmh;
                    }
                    store(b, rr, limb_reduce4(c0, p), limb_reduce4(c1, p));
                }
            });
        };
        if (fd) run(std::true_type{});
        else run(std::false_type{});
    } else {
        // other primes: 128-bit sums of full products, one reduction per output
        u64 kb[RR][K], ka[RR][K];
#pragma unroll
        for (int rr = 0; rr < RR; ++rr)
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int n = (voff_o[rr] >> 3) % N;
                kb[rr][j] = __builtin_nontemporal_load(&key[rr][((long)(j * 2 + 0) * np + pt) * N + n]);
                ka[rr][j] = __builtin_nontemporal_load(&key[rr][((long)(j * 2 + 1) * np + pt) * N + n]);
            }
        auto run = [&](auto fold_tag) {
            constexpr bool FOLD = decltype(fold_tag)::value;
            batch(fold_tag, [&](int b, const u64 (&x)[K], u64 fx) {
#pragma unroll
                for (int rr = 0; rr < RR; ++rr) {
                    Acc a0, a1;
                    acc_zero(a0);
                    acc_zero(a1);
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        acc_mac(a0, x[j], kb[rr][j]);
                        acc_mac(a1, x[j], ka[rr][j]);
                    }
                    if constexpr (FOLD) acc_mac(a0, fx, fm);
                    store(b, rr, acc_reduce(a0, p), acc_reduce(a1, p));
                }
            });
        };
        if (fd) run(std::true_type{});
        else run(std::false_type{});
    }
}

// Waves per SIMD each key-product kernel is compiled for (its register budget: 512 / waves).
template <int CLS, int RR>
constexpr int kKeyipWaves = CLS == KIP_FP ? (RR <= 4 ? 3 : 2) : (RR <= 2 ? 3 : 2);

#define CTL_KEYIP_KERNEL(NAME, CLS)                                                                        \
    template <int K, int RR>                                                                               \
    __global__ void __launch_bounds__(256, (kKeyipWaves<CLS, RR>))                                         \
    NAME(const u64 *__restrict__ digits, long db, long dr, KeyList keys, u64 *__restrict__ out, long ob,    \
         KeyFold fold, RowSet rows, int B, int R, int nq, int logn, int xcd_order,                         \
         const PrimeConst *__restrict__ pcs) {                                                             \
        keyip_body<K, RR, CLS>(digits, db, dr, keys, out, ob, fold, rows, B, R, nq, logn, xcd_order, pcs); \
    }
CTL_KEYIP_KERNEL(k_keyip_fp, KIP_FP)
CTL_KEYIP_KERNEL(k_keyip_limb, KIP_LIMB)
CTL_KEYIP_KERNEL(k_keyip, KIP_WIDE)
#undef CTL_KEYIP_KERNEL

// Baby-step MAC of Eq. (1): inner[b][k2][c][i] = sum_{j < t1} pt[k2 t1 + j][i] * rot_j(ct_b)[c][i]
// with rot_0 = ct itself (ct_b at ct + b ct_sb, [2][K][N]) and rot_j, j >= 1, at rot + b rot_sb +
// (j - 1) 2 K N. K = `k` residue rows per polynomial (with the baby steps kept over Q*P the last
// row is mod P); row i = pl.idx[y] has prime pl.prime[y].
// Per coefficient this is a (t2 x t1) by (t1 x 2B) modular matrix product. A workgroup covers 64
// consecutive coefficients of one prime for up to 16 (FP64) or 8 (integer) ciphertexts
// (threadIdx.y); each thread keeps
// KC giant-step accumulators per polynomial, so every rotated ciphertext word is read once per
// KC-chunk. The plaintext words of JB baby steps are staged in LDS and shared by the workgroup's
// ciphertexts (k_mac: per barrier pair, the ciphertext words of those JB steps loaded first;
// k_mac_fp and k_mac_limb: pipelined, see below).
// grid: x = N / 64 tiles, y = prime (from a PrimeList), z = ceil(B / blockDim.y) ciphertext
// groups times t2 / KC chunks (a grid dimension, so that small batches still fill the GPU).
constexpr int kMacJB = 4;

// The FP64 and integer forms are separate kernels launched over their own primes (PrimeList,
// grid y), so that the FP64 one is not held to the register budget of 128-bit accumulators.
//
// k_mac_fp and k_mac_limb are software-pipelined over JB-chunks of baby steps. Before a chunk is
// multiplied, this wave's rows of the next chunk's plaintext words are loaded into registers; they
// go to the other of two LDS buffers afterwards, so each chunk costs one barrier. Each rotated
// ciphertext word, once consumed, has its register refilled with the word at the same position
// of the next chunk. Staging row r of a chunk (r = jj KC + kk, 64 words) belongs to the wave of
// threadIdx.y = r mod blockDim.y; with 8 or more ciphertexts per workgroup that is at most
// kMacStage(KC) rows per wave, and smaller workgroups stage their remaining rows after the
// multiplications.
template <int KC>
constexpr int kMacStage = (kMacJB * KC + 7) / 8;

template <int KC>
__global__ void __launch_bounds__(1024)
k_mac_fp(const u64 *__restrict__ ct, long ct_sb, const u64 *__restrict__ rot, long rot_sb,
         const u64 *__restrict__ bank, u64 *__restrict__ inner, int B, int k, int t1, int t2, int logn,
         PrimeList pl, const PrimeConst *__restrict__ pcs) {
    constexpr int kSt = kMacStage<KC>;
    __shared__ double wd[2][kMacJB * KC * 64];
    const int nl = threadIdx.x, bl = __builtin_amdgcn_readfirstlane(threadIdx.y), by = blockDim.y;
    const int i = pl.idx[blockIdx.y];
    const long N = 1L << logn, kn = (long)k * N;
    const long n0 = (long)blockIdx.x * 64;
    const int nbz = (B + by - 1) / by;              // grid z = ciphertext groups x KC-chunks
    const int b = (blockIdx.z % nbz) * by + bl;
    const int kc0 = (blockIdx.z / nbz) * KC;
    const bool live = b < B;
    const PrimeConst p = pcs[pl.prime[blockIdx.y]];
    const u64 *ct_b = ct + (long)(live ? b : 0) * ct_sb + i * N + n0 + nl;
    const u64 *rot_b = rot + (long)(live ? b : 0) * rot_sb + i * N + n0 + nl;
    const u64 *bk = bank + (long)kc0 * t1 * kn + i * N + n0 + nl;
    // plaintext word of staging row r (wave-uniform) of the chunk starting at baby step j0
    auto bank_row = [&](int j0, int r) -> u64 { return bk[((long)(r % KC) * t1 + j0 + r / KC) * kn]; };
    double acc[KC][2];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) acc[kk][0] = acc[kk][1] = 0.0;
    u64 xr[kMacJB][2];
    {
        const int jn = t1 < kMacJB ? t1 : kMacJB;
#pragma unroll
        for (int jj = 0; jj < kMacJB; ++jj) {
            if (jj < jn) {
                const u64 *src = jj == 0 ? ct_b : rot_b + (long)(jj - 1) * 2 * kn;
                xr[jj][0] = __builtin_nontemporal_load(&src[0]);
                xr[jj][1] = __builtin_nontemporal_load(&src[kn]);
            }
        }
        for (int r = bl; r < jn * KC; r += by) wd[0][r * 64 + nl] = u64_to_fp(bank_row(0, r));
    }
    __syncthreads();
    int buf = 0;
    for (int j0 = 0; j0 < t1; j0 += kMacJB, buf ^= 1) {
        const int jn = t1 - j0 < kMacJB ? t1 - j0 : kMacJB;
        const int j1 = j0 + kMacJB;
        const int jn1 = j1 >= t1 ? 0 : (t1 - j1 < kMacJB ? t1 - j1 : kMacJB);
        const int rows1 = jn1 * KC;
        u64 bs[kSt];
#pragma unroll
        for (int s = 0; s < kSt; ++s) {
            const int r = bl + s * by;
            bs[s] = bank_row(j1 < t1 ? j1 : j0, r < rows1 ? r : 0);   // unconditional: no early wait
        }
        const double *w_l = wd[buf];
#pragma unroll
        for (int jj = 0; jj < kMacJB; ++jj) {
            if (jj < jn) {
                const double x0 = u64_to_fp(live ? xr[jj][0] : 0), x1 = u64_to_fp(live ? xr[jj][1] : 0);
                if (jj < jn1) {                  // uniform; rot_b of a spare thread is a valid row
                    const u64 *src = rot_b + (long)(j1 + jj - 1) * 2 * kn;
                    xr[jj][0] = __builtin_nontemporal_load(&src[0]);
                    xr[jj][1] = __builtin_nontemporal_load(&src[kn]);
                }
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const double w = w_l[(jj * KC + kk) * 64 + nl];
                    acc[kk][0] += fp_mul(x0, w, p.qd, p.qinv);
                    acc[kk][1] += fp_mul(x1, w, p.qd, p.qinv);
                }
            }
        }
        double *w_n = wd[buf ^ 1];
#pragma unroll
        for (int s = 0; s < kSt; ++s) {
            const int r = bl + s * by;
            if (r < rows1) w_n[r * 64 + nl] = u64_to_fp(bs[s]);
        }
        for (int r = bl + kSt * by; r < rows1; r += by) w_n[r * 64 + nl] = u64_to_fp(bank_row(j1, r));
        __syncthreads();
    }
    if (live) {
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            u64 *o = inner + ((long)b * t2 + kc0 + kk) * 2 * kn + i * N + n0 + nl;
            __builtin_nontemporal_store(fp_to_u64(acc[kk][0], p.qd, p.qinv), &o[0]);
            __builtin_nontemporal_store(fp_to_u64(acc[kk][1], p.qd, p.qinv), &o[kn]);
        }
    }
}

template <int KC>
__global__ void __launch_bounds__(512)
k_mac(const u64 *__restrict__ ct, long ct_sb, const u64 *__restrict__ rot, long rot_sb,
      const u64 *__restrict__ bank, u64 *__restrict__ inner, int B, int k, int t1, int t2, int logn,
      PrimeList pl, const PrimeConst *__restrict__ pcs) {
    __shared__ u64 wt[kMacJB * KC * 64];
    const int nl = threadIdx.x, bl = threadIdx.y;
    const int tid = bl * 64 + nl, nthr = 64 * blockDim.y;
    const int i = pl.idx[blockIdx.y];
    const long N = 1L << logn, kn = (long)k * N;
    const long n0 = (long)blockIdx.x * 64;
    const int nbz = (B + blockDim.y - 1) / blockDim.y;   // grid z = ciphertext groups x KC-chunks
    const int b = (blockIdx.z % nbz) * blockDim.y + bl;
    const int kc0 = (blockIdx.z / nbz) * KC;
    const bool live = b < B;
    const PrimeConst p = pcs[pl.prime[blockIdx.y]];
    const u64 *ct_b = ct + (long)(live ? b : 0) * ct_sb + i * N + n0 + nl;
    const u64 *rot_b = rot + (long)(live ? b : 0) * rot_sb + i * N + n0 + nl;
    {
        Acc acc[KC][2];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) { acc_zero(acc[kk][0]); acc_zero(acc[kk][1]); }
        for (int j0 = 0; j0 < t1; j0 += kMacJB) {
            const int jn = t1 - j0 < kMacJB ? t1 - j0 : kMacJB;
            u64 x[kMacJB][2];
#pragma unroll
            for (int jj = 0; jj < kMacJB; ++jj) {
                const int j = j0 + jj;
                if (live && jj < jn) {
                    const u64 *src = j == 0 ? ct_b : rot_b + (long)(j - 1) * 2 * kn;
                    x[jj][0] = src[0];
                    x[jj][1] = src[kn];
                } else {
                    x[jj][0] = x[jj][1] = 0;
                }
            }
            __syncthreads();
            for (int e = tid; e < jn * KC * 64; e += nthr) {
                const int jj = e / (KC * 64), kk = (e / 64) % KC;
                wt[e] = bank[((long)(kc0 + kk) * t1 + j0 + jj) * kn + i * N + n0 + (e & 63)];
            }
            __syncthreads();
#pragma unroll
            for (int jj = 0; jj < kMacJB; ++jj) {
                if (jj < jn) {
#pragma unroll
                    for (int kk = 0; kk < KC; ++kk) {
                        const u64 w = wt[(jj * KC + kk) * 64 + nl];
                        acc_mac(acc[kk][0], w, x[jj][0]);
                        acc_mac(acc[kk][1], w, x[jj][1]);
                    }
                }
            }
        }
        if (live) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                u64 *o = inner + ((long)b * t2 + kc0 + kk) * 2 * kn + i * N + n0 + nl;
                o[0] = acc_reduce(acc[kk][0], p);
                o[kn] = acc_reduce(acc[kk][1], p);
            }
        }
    }
}

// The integer-prime MAC with 30-bit limbs, for rows whose prime is below 2^60 (every residue
// then splits as x = xh 2^30 + xl with xh, xl < 2^30). A product x w is four 30 x 30-bit products
// accumulated by v_mad_u64_u32 without carries into three 64-bit column sums of weights 1, 2^30
// and 2^60 (c[1] takes both cross products). Every 8 terms the columns are normalized (c0, c1 <
// 2^30, c2 < 2^62), which keeps each below 2^64 for the next 8: c0 < 2^30 + 8 2^60,
// c1 < 2^30 + 16 (2^30 - 1)^2, c2 < 2^62 + 8 2^60 + 2^34. Once per output the 128-bit value
// c0 + c1 2^30 + c2 2^60 is reduced mod q. Same staging and outputs as k_mac; plaintext
// words are staged split into their limbs, wl | wh 2^32, so that the waves reading the LDS copy
// find the limbs as register halves. grid: x = N / 64 tiles times t2 / KC chunks (tile-major in
// blocks of 8 tiles, see below), y = prime, z = ceil(B / blockDim.y) ciphertext groups.
template <int KC>
__global__ void __launch_bounds__(512)
k_mac_limb(const u64 *__restrict__ ct, long ct_sb, const u64 *__restrict__ rot, long rot_sb,
           const u64 *__restrict__ bank, u64 *__restrict__ inner, int B, int k, int t1, int t2, int logn,
           PrimeList pl, const PrimeConst *__restrict__ pcs) {
    constexpr int kSt = kMacStage<KC>;
    __shared__ u64 wt[2][kMacJB * KC * 64];
    const int nl = threadIdx.x, bl = __builtin_amdgcn_readfirstlane(threadIdx.y), by = blockDim.y;
    const int i = pl.idx[blockIdx.y];
    const long N = 1L << logn, kn = (long)k * N;
    // grid x = tiles x KC-chunks, the chunks of one tile 8 workgroups apart: they run on one XCD
    // at about the same time, so all but the first read the tile's ciphertext words from its L2
    const int nch = t2 / KC, hx = (int)blockIdx.x >> 3, lx = (int)blockIdx.x & 7;
    const long n0 = (long)(nch == 1 ? (int)blockIdx.x : (hx / nch) * 8 + lx) * 64;
    const int kc0 = nch == 1 ? 0 : (hx % nch) * KC;
    const int b = (int)blockIdx.z * by + bl;        // grid z = ciphertext groups
    const bool live = b < B;
    const PrimeConst p = pcs[pl.prime[blockIdx.y]];
    const u64 *ct_b = ct + (long)(live ? b : 0) * ct_sb + i * N + n0 + nl;
    const u64 *rot_b = rot + (long)(live ? b : 0) * rot_sb + i * N + n0 + nl;
    const u64 *bk = bank + (long)kc0 * t1 * kn + i * N + n0 + nl;
    auto bank_row = [&](int j0, int r) -> u64 { return bk[((long)(r % KC) * t1 + j0 + r / KC) * kn]; };
    auto split = [](u64 w) -> u64 { return (w & kM30) | ((w >> 30) << 32); };
    u64 c[KC][2][3];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
        for (int q = 0; q < 2; ++q) c[kk][q][0] = c[kk][q][1] = c[kk][q][2] = 0;
    u64 xr[kMacJB][2];
    {
        const int jn = t1 < kMacJB ? t1 : kMacJB;
#pragma unroll
        for (int jj = 0; jj < kMacJB; ++jj) {
            if (live && jj < jn) {
                const u64 *src = jj == 0 ? ct_b : rot_b + (long)(jj - 1) * 2 * kn;
                xr[jj][0] = __builtin_nontemporal_load(&src[0]);
                xr[jj][1] = __builtin_nontemporal_load(&src[kn]);
            }
        }
        for (int r = bl; r < jn * KC; r += by) wt[0][r * 64 + nl] = split(bank_row(0, r));
    }
    __syncthreads();
    int since = 0;                               // terms added since the last normalization
    int buf = 0;
    for (int j0 = 0; j0 < t1; j0 += kMacJB, buf ^= 1) {
        const int jn = t1 - j0 < kMacJB ? t1 - j0 : kMacJB;
        const int j1 = j0 + kMacJB;
        const int jn1 = j1 >= t1 ? 0 : (t1 - j1 < kMacJB ? t1 - j1 : kMacJB);
        const int rows1 = jn1 * KC;
        u64 bs[kSt];
#pragma unroll
        for (int s = 0; s < kSt; ++s) {
            const int r = bl + s * by;
            bs[s] = bank_row(j1 < t1 ? j1 : j0, r < rows1 ? r : 0);   // unconditional: no early wait
        }
        if (since + jn > 8) {                    // uniform: keep every column below 2^64
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                limb_normalize(c[kk][0], p);
                limb_normalize(c[kk][1], p);
            }
            since = 0;
        }
        const u64 *w_l = wt[buf];
#pragma unroll
        for (int jj = 0; jj < kMacJB; ++jj) {
            if (jj < jn) {
                const u64 x0 = live ? xr[jj][0] : 0, x1 = live ? xr[jj][1] : 0;
                const u32 xl[2] = {(u32)x0 & (u32)kM30, (u32)x1 & (u32)kM30};
                const u32 xh[2] = {(u32)(x0 >> 30), (u32)(x1 >> 30)};
                if (jj < jn1) {                  // uniform; rot_b of a spare thread is a valid row
                    const u64 *src = rot_b + (long)(j1 + jj - 1) * 2 * kn;
                    xr[jj][0] = __builtin_nontemporal_load(&src[0]);
                    xr[jj][1] = __builtin_nontemporal_load(&src[kn]);
                }
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const u64 w = w_l[(jj * KC + kk) * 64 + nl];
                    const u32 wl = (u32)w, wh = (u32)(w >> 32);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        c[kk][q][0] += (u64)xl[q] * wl;
                        c[kk][q][1] += (u64)xl[q] * wh;
                        c[kk][q][1] += (u64)xh[q] * wl;
                        c[kk][q][2] += (u64)xh[q] * wh;
                    }
                }
            }
        }
        since += jn;
        u64 *w_n = wt[buf ^ 1];
#pragma unroll
        for (int s = 0; s < kSt; ++s) {
            const int r = bl + s * by;
            if (r < rows1) w_n[r * 64 + nl] = split(bs[s]);
        }
        for (int r = bl + kSt * by; r < rows1; r += by) w_n[r * 64 + nl] = split(bank_row(j1, r));
        __syncthreads();
    }
    if (live) {
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            u64 *o = inner + ((long)b * t2 + kc0 + kk) * 2 * kn + i * N + n0 + nl;
            __builtin_nontemporal_store(limb_reduce(c[kk][0], p), &o[0]);
            __builtin_nontemporal_store(limb_reduce(c[kk][1], p), &o[kn]);
        }
    }
}

// The same MAC for batches of one or two ciphertexts: there is nothing to share a staged plaintext
// word with, so each thread reads its plaintext words straight from memory (coalesced across the
// coefficients of a wave), with no LDS and no barriers, and FP64 and integer primes go in one
// launch (the branch is uniform per workgroup). Plaintext words are read once per launch, so their
// loads are non-temporal: they stay out of L2, which keeps the rotated ciphertext words the
// giant-step chunks share. grid: x = N / 64 tiles, y = residue row
// (PrimeList), z = B t2 / KC.
template <int KC>
__global__ void __launch_bounds__(64)
k_mac_direct(const u64 *__restrict__ ct, long ct_sb, const u64 *__restrict__ rot, long rot_sb,
             const u64 *__restrict__ bank, u64 *__restrict__ inner, int B, int k, int t1, int t2, int logn,
             PrimeList pl, const PrimeConst *__restrict__ pcs) {
    const int nl = threadIdx.x, i = pl.idx[blockIdx.y];
    const long N = 1L << logn, kn = (long)k * N;
    const long n0 = (long)blockIdx.x * 64;
    const int b = blockIdx.z % B, kc0 = (blockIdx.z / B) * KC;
    const PrimeConst p = pcs[pl.prime[blockIdx.y]];
    const u64 *ct_b = ct + (long)b * ct_sb + i * N + n0 + nl;
    const u64 *rot_b = rot + (long)b * rot_sb + i * N + n0 + nl;
    const u64 *bk = bank + i * N + n0 + nl;
    if (p.fp) {
        double acc[KC][2];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) acc[kk][0] = acc[kk][1] = 0.0;
        for (int j = 0; j < t1; ++j) {
            const u64 *src = j == 0 ? ct_b : rot_b + (long)(j - 1) * 2 * kn;
            const double x0 = u64_to_fp(src[0]), x1 = u64_to_fp(src[kn]);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const double w = u64_to_fp(__builtin_nontemporal_load(&bk[((long)(kc0 + kk) * t1 + j) * kn]));
                acc[kk][0] += fp_mul(x0, w, p.qd, p.qinv);
                acc[kk][1] += fp_mul(x1, w, p.qd, p.qinv);
            }
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            u64 *o = inner + ((long)b * t2 + kc0 + kk) * 2 * kn + i * N + n0 + nl;
            o[0] = fp_to_u64(acc[kk][0], p.qd, p.qinv);
            o[kn] = fp_to_u64(acc[kk][1], p.qd, p.qinv);
        }
        return;
    }
    Acc acc[KC][2];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) { acc_zero(acc[kk][0]); acc_zero(acc[kk][1]); }
    for (int j = 0; j < t1; ++j) {
        const u64 *src = j == 0 ? ct_b : rot_b + (long)(j - 1) * 2 * kn;
        const u64 x0 = src[0], x1 = src[kn];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const u64 w = __builtin_nontemporal_load(&bk[((long)(kc0 + kk) * t1 + j) * kn]);
            acc_mac(acc[kk][0], w, x0);
            acc_mac(acc[kk][1], w, x1);
        }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        u64 *o = inner + ((long)b * t2 + kc0 + kk) * 2 * kn + i * N + n0 + nl;
        o[0] = acc_reduce(acc[kk][0], p);
        o[kn] = acc_reduce(acc[kk][1], p);
    }
}

// out[b][c][i] = a[b][c][i] + sum_{s < S} terms[b][s][c][i]; each operand ct-shaped [2][k][N].
__global__ void __launch_bounds__(256)
k_add_terms(const u64 *__restrict__ a, long a_sb, const u64 *__restrict__ terms, long t_sb, long t_ss,
            int S, u64 *__restrict__ out, int k, int logn, const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;   // over 2 k N
    const int b = blockIdx.y;
    const int i = (int)((idx / N) % k);
    const u64 q = pcs[i].q;
    u64 s = a[b * a_sb + idx];
    for (int t = 0; t < S; ++t) s = add_mod(s, terms[b * t_sb + t * t_ss + idx], q);
    out[(long)b * 2 * k * N + idx] = s;
}

// out[b][c][t] = P in[b][c][t] mod q_t (t < k) and 0 for the row mod P (t = k).
// grid: x = N / 256, y = 2 (k + 1), z = B.
__global__ void __launch_bounds__(256)
k_times_p(const u64 *__restrict__ in, u64 *__restrict__ out, long o_sb, int k, int nq, int logn,
          const PrimeConst *__restrict__ pcs, const CrossConst *__restrict__ cross) {
    const long N = 1L << logn;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y / (k + 1), t = blockIdx.y % (k + 1), b = blockIdx.z;
    u64 v = 0;
    if (t < k) {
        const PrimeConst p = pcs[t];
        v = mul_mod(in[((long)b * 2 * k + (long)c * k + t) * N + n], cross[t * kMaxMods + nq].qj_mod_qi, p);
    }
    out[b * o_sb + ((long)c * (k + 1) + t) * N + n] = v;
}

// out[b][c][t] = base[b][c][t] (or 0) + sum_{r < R} src[b][r][c][t] gathered through sigma_{gal[r]},
// for the polynomials c set in mask (others copy base). kk residues per polynomial; with ext the
// last one is mod P (prime index nq). grid: x = N / 256, y = 2 kk, z = B.
__global__ void __launch_bounds__(256)
k_sum_gather(u64 *__restrict__ out, long o_sb, const u64 *__restrict__ base, long ba_sb,
             const u64 *__restrict__ src, long s_sb, long s_sr, int R, int kk, int ext, int mask, GalList gal,
             int nq, int logn, const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y / kk, t = blockIdx.y % kk, b = blockIdx.z;
    const int pi = (ext && t == kk - 1) ? nq : t;
    const u64 q = pcs[pi].q;
    const long off = ((long)c * kk + t) * N;
    u64 s = base ? base[b * ba_sb + off + n] : 0;
    if ((mask >> c) & 1) {
        for (int r = 0; r < R; ++r) {
            const u64 g = gal.g[r];
            s = add_mod(s, src[b * s_sb + r * s_sr + off + (g == 1 ? n : galois_src(n, g, logn))], q);
        }
    }
    out[b * o_sb + off + n] = s;
}

// (a0, a1) x (b0, b1) -> (a0 b0, a0 b1 + a1 b0, a1 b1): a, b [B][2][k][N], out [B][3][k][N].
__global__ void __launch_bounds__(256)
k_tensor(const u64 *__restrict__ a, const u64 *__restrict__ bb, u64 *__restrict__ out, int k, int logn,
         const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn, kn = (long)k * N;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;   // over k N
    const int b = blockIdx.y;
    const PrimeConst p = pcs[idx / N];
    const u64 a0 = a[b * 2 * kn + idx], a1 = a[b * 2 * kn + kn + idx];
    const u64 b0 = bb[b * 2 * kn + idx], b1 = bb[b * 2 * kn + kn + idx];
    u64 *o = out + b * 3 * kn + idx;
    o[0] = mul_mod(a0, b0, p);
    o[kn] = add_mod(mul_mod(a0, b1, p), mul_mod(a1, b0, p), p.q);
    o[2 * kn] = mul_mod(a1, b1, p);
}

// out[b][c][i] = in[b][c][i] * mul_i + (c == 0 ? add_i : 0) mod q_i for the first k_out of the
// k_in residues of each polynomial (dropping the others lowers the level, keeping the value).
__global__ void __launch_bounds__(256)
k_affine(const u64 *in, u64 *out, int k_in, int k_out, AffineConst ac, int logn,
         const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;   // over 2 k_out N
    const int b = blockIdx.y;
    const int c = (int)(idx / ((long)k_out * N)), i = (int)((idx / N) % k_out);
    const long x = idx % N;
    const PrimeConst p = pcs[i];
    const u64 v = in[((long)b * 2 * k_in + (long)c * k_in + i) * N + x];
    u64 r = red2(shoup_lazy(v, ac.mul[i], ac.muls[i], p.q, p.qn), p.q);
    if (c == 0) r = add_mod(r, ac.add[i], p.q);
    out[((long)b * 2 * k_out + (long)c * k_out + i) * N + x] = r;
}

// Key-switching key body: key[j][0][i] = -a s + e (+ [P]_{q_i} s'_i when i == j); a already at
// key[j][1][i]; e: [nq][np][N] NTT form; s: [np][N]; sp (s' over q_0..q_{nq-1}) either given or
// sigma_g(s) by gather (g != 0) or s^2 (g == 0).
__global__ void __launch_bounds__(256)
k_ksk_body(u64 *__restrict__ key, const u64 *__restrict__ e, const u64 *__restrict__ s, u64 g,
           int nq, int logn, const PrimeConst *__restrict__ pcs, const CrossConst *__restrict__ cross) {
    const int N = 1 << logn, np = nq + 1;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int i = blockIdx.y, j = blockIdx.z;
    const PrimeConst p = pcs[i];
    const long o0 = ((long)(j * 2 + 0) * np + i) * N + n;
    const long o1 = ((long)(j * 2 + 1) * np + i) * N + n;
    const u64 si = s[(long)i * N + n];
    u64 b = sub_mod(e[((long)j * np + i) * N + n], mul_mod(key[o1], si, p), p.q);
    if (i == j) {
        u64 sp;
        if (g == 0) sp = mul_mod(si, si, p);
        else sp = s[(long)i * N + galois_src(n, g, logn)];
        const u64 pm = cross[i * kMaxMods + nq].qj_mod_qi;      // P mod q_i
        b = add_mod(b, mul_mod(pm, sp, p), p.q);
    }
    key[o0] = b;
}

// Public key: pk[0][i] = -a s + e with a at pk[1][i]; e: [nq][N] NTT form.
__global__ void __launch_bounds__(256)
k_pk_body(u64 *__restrict__ pk, const u64 *__restrict__ e, const u64 *__restrict__ s, int nq, int logn,
          const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn;
    const int n = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
    const PrimeConst p = pcs[i];
    const long o = (long)i * N + n;
    pk[o] = sub_mod(e[o], mul_mod(pk[(long)nq * N + o], s[o], p), p.q);
}

// Encryption: in = [4][nq][N] NTT form of (v, e0, e1, m); ct = (v b + e0 + m, v a + e1).
__global__ void __launch_bounds__(256)
k_encrypt(const u64 *__restrict__ pk, const u64 *__restrict__ in, u64 *__restrict__ ct, int nq, int logn,
          const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn, qn = (long)nq * N;
    const int n = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
    const PrimeConst p = pcs[i];
    const long o = (long)i * N + n;
    const u64 v = in[o], e0 = in[qn + o], e1 = in[2 * qn + o], m = in[3 * qn + o];
    ct[o] = add_mod(add_mod(mul_mod(v, pk[o], p), e0, p.q), m, p.q);
    ct[qn + o] = add_mod(mul_mod(v, pk[qn + o], p), e1, p.q);
}

// Decryption product c0 + c1 s for k primes (NTT form): ct [2][k][N], s [np][N], out [k][N].
__global__ void __launch_bounds__(256)
k_dec_mul(const u64 *__restrict__ ct, const u64 *__restrict__ s, u64 *__restrict__ out, int k, int logn,
          const PrimeConst *__restrict__ pcs) {
    const long N = 1L << logn, kn = (long)k * N;
    const int n = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
    const PrimeConst p = pcs[i];
    const long o = (long)i * N + n;
    out[o] = add_mod(ct[o], mul_mod(ct[kn + o], s[o], p), p.q);
}

// ---------------------------------------------------------------- launchers
template <typename F>
static hipError_t set_lds(F f, int bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int LOGN>
static hipError_t prepare_all() {
    const int b = lds_words<LOGN>() * 8;
    hipError_t e;
    if ((e = set_lds(k_ntt_fwd<LOGN>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_ntt_inv<LOGN>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_modup<LOGN>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_drop<LOGN>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpNtt, true>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpNtt, false>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_inv_loop<LOGN, OpNtt, true>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_inv_loop<LOGN, OpNtt, false>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpModup, true>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpModup, false>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpDrop, true>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpDrop, false>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpDropRescale, true>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_loop<LOGN, OpDropRescale, false>, b)) != hipSuccess) return e;
    if ((e = set_lds(k_fwd_one<LOGN, OpDropRescale>, b)) != hipSuccess) return e;
    return set_lds(k_int_ntt<LOGN>, b);
}

// ---------------------------------------------------------------- vector ALU issue-rate probe
// KIND 0: 32-bit add, 1: 32-bit multiply (low half), 2: v_mad_u64_u32 (32 x 32 + 64), 3: FP64 fma.
// Each thread runs kProbeChains chains, each step of which takes its neighbour's previous value
// (so no step can be folded or hoisted), for `iters` iterations of 8 steps; the result is stored.
constexpr int kProbeChains = 8;

template <int KIND>
__global__ void __launch_bounds__(256) k_probe(int iters, u64 seed, u64 *__restrict__ out) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    u64 x[kProbeChains];
    double d[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
        x[c] = (seed + (u64)gid * 0x9E3779B97F4A7C15ull + (u64)c * 0xBF58476D1CE4E5B9ull) | 1ull;
        d[c] = 1.0 + (double)((x[c] >> 11) & 1023) * 0x1p-12;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if constexpr (KIND == 3) {
                double nd[kProbeChains];
#pragma unroll
                for (int c = 0; c < kProbeChains; ++c) nd[c] = __fma_rn(d[c], -0.5, d[(c + 1) % kProbeChains]);
#pragma unroll
                for (int c = 0; c < kProbeChains; ++c) d[c] = nd[c];
            } else {
                u64 nx[kProbeChains];
#pragma unroll
                for (int c = 0; c < kProbeChains; ++c) {
                    const u64 y = x[(c + 1) % kProbeChains];
                    if constexpr (KIND == 0) nx[c] = (u32)x[c] + (u32)y;
                    else if constexpr (KIND == 1) nx[c] = (u32)x[c] * (u32)y;
                    else nx[c] = (u64)(u32)x[c] * (u32)(y >> 32) + x[c];
                }
#pragma unroll
                for (int c = 0; c < kProbeChains; ++c) x[c] = nx[c];
            }
        }
    }
    u64 acc = 0;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) acc ^= KIND == 3 ? (u64)__double_as_longlong(d[c]) : x[c];
    out[gid] = acc;
}

void launch_probe(int kind, int iters, u64 seed, u64 *out, int blocks, hipStream_t st) {
    const dim3 grid((unsigned)blocks), blk(256);
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_probe<0>, grid, blk, 0, st, iters, seed, out); break;
        case 1: hipLaunchKernelGGL(k_probe<1>, grid, blk, 0, st, iters, seed, out); break;
        case 2: hipLaunchKernelGGL(k_probe<2>, grid, blk, 0, st, iters, seed, out); break;
        default: hipLaunchKernelGGL(k_probe<3>, grid, blk, 0, st, iters, seed, out); break;
    }
}

// Scratch of the entry point that allocates nothing. Host code never passes `scratch` itself to
// a kernel (in host code the name is a stand-in, not a device address): it passes the address
// hipGetSymbolAddress returns for the current device, looked up once per device.
static __device__ __align__(256) u64 scratch[kScratchWords];

hipError_t scratch_device_address(int device, u64 **out) {
    static std::mutex mu;
    static std::map<int, u64 *> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<u64 *>(p);
    *out = static_cast<u64 *>(p);
    return hipSuccess;
}

hipError_t kernels_prepare(int logn) {
    switch (logn) {
        case 12: return prepare_all<12>();
        case 13: return prepare_all<13>();
        case 14: return prepare_all<14>();
        default: return hipErrorInvalidValue;
    }
}


void launch_ntt(int logn, bool inverse, const u64 *in, const ResMap &imap, u64 *out, const ResMap &omap,
                int count, const Tables &tab, const Knobs &kn, hipStream_t st, u64 *split_tmp, int cls) {
    if (count <= 0) return;
    if (split_tmp) {
        const OpNtt op{in, imap, out, omap, logn};
        if (inverse) launch_split_inv(logn, op, split_tmp, count, tab, st);
        else launch_split_fwd(logn, op, split_tmp, count, tab, st);
        return;
    }
    if (use_loop(count, imap.prime, imap.per, tab, kn)) {
        const OpNtt op{in, imap, out, omap, logn};
        if (inverse) launch_loop<true>(logn, op, imap.prime, imap.per, count, tab, st, cls);
        else launch_loop<false>(logn, op, imap.prime, imap.per, count, tab, st, cls);
        return;
    }
    const dim3 grid(count), blk = ntt_block(logn);
    const size_t sh = ntt_lds(logn);
    if (inverse) {
        switch (logn) {
            case 12: hipLaunchKernelGGL(k_ntt_inv<12>, grid, blk, sh, st, in, imap, out, omap, tab); break;
            case 13: hipLaunchKernelGGL(k_ntt_inv<13>, grid, blk, sh, st, in, imap, out, omap, tab); break;
            default: hipLaunchKernelGGL(k_ntt_inv<14>, grid, blk, sh, st, in, imap, out, omap, tab); break;
        }
    } else {
        switch (logn) {
            case 12: hipLaunchKernelGGL(k_ntt_fwd<12>, grid, blk, sh, st, in, imap, out, omap, tab); break;
            case 13: hipLaunchKernelGGL(k_ntt_fwd<13>, grid, blk, sh, st, in, imap, out, omap, tab); break;
            default: hipLaunchKernelGGL(k_ntt_fwd<14>, grid, blk, sh, st, in, imap, out, omap, tab); break;
        }
    }
}

void launch_modup(int logn, const u64 *coef, const u64 *d, const ResMap &dmap, u64 *digits, int groups, int k,
                  int nq, const Tables &tab, const Knobs &kn, hipStream_t st, u64 *split_tmp, int cls) {
    if (groups <= 0) return;
    if (split_tmp) {
        launch_split_fwd(logn, OpModup{coef, d, dmap, digits, k, nq, logn}, split_tmp, groups * k * (k + 1), tab, st);
        return;
    }
    const int units = groups * k, xo = kn.ntt_xcd ? 1 : 0;
    int prime[kMaxMods];
    modup_primes(k, nq, prime);
    if (use_loop(units * (k + 1), prime, k + 1, tab, kn)) {
        launch_loop<false>(logn, OpModup{coef, d, dmap, digits, k, nq, logn}, prime, k + 1, units * (k + 1), tab, st,
                           cls);
        return;
    }
    const dim3 grid(xo ? ((units + 7) / 8) * 8 * (k + 1) : units * (k + 1)), blk = ntt_block(logn);
    const size_t sh = ntt_lds(logn);
    switch (logn) {
        case 12: hipLaunchKernelGGL(k_modup<12>, grid, blk, sh, st, coef, d, dmap, digits, k, nq, units, xo, tab); break;
        case 13: hipLaunchKernelGGL(k_modup<13>, grid, blk, sh, st, coef, d, dmap, digits, k, nq, units, xo, tab); break;
        default: hipLaunchKernelGGL(k_modup<14>, grid, blk, sh, st, coef, d, dmap, digits, k, nq, units, xo, tab); break;
    }
}

void launch_drop(int logn, const u64 *x, const u64 *last, u64 *out, int groups, int k, int drop,
                 const DropAdd &add, const Tables &tab, const Knobs &kn, hipStream_t st, const GrpMap *xmap,
                 u64 *split_tmp, int cls) {
    if (groups <= 0) return;
    const long N = 1L << logn;
    const GrpMap xm = xmap ? *xmap : GrpMap{0, (k + 1) * N, 0, 1};
    if (split_tmp) {
        launch_split_fwd(logn, OpDrop{x, xm, last, out, k, drop, logn, add}, split_tmp, groups * k, tab, st);
        return;
    }
    int prime[kMaxMods];
    drop_primes(k, prime);
    if (use_loop(groups * k, prime, k, tab, kn)) {
        launch_loop<false>(logn, OpDrop{x, xm, last, out, k, drop, logn, add}, prime, k, groups * k, tab, st, cls);
        return;
    }
    const int xo = kn.ntt_xcd ? 1 : 0;
    const dim3 grid(xo ? ((groups + 7) / 8) * 8 * k : groups * k), blk = ntt_block(logn);
    const size_t sh = ntt_lds(logn);
    switch (logn) {
        case 12: hipLaunchKernelGGL(k_drop<12>, grid, blk, sh, st, x, xm, last, out, k, drop, groups, xo, add, tab); break;
        case 13: hipLaunchKernelGGL(k_drop<13>, grid, blk, sh, st, x, xm, last, out, k, drop, groups, xo, add, tab); break;
        default: hipLaunchKernelGGL(k_drop<14>, grid, blk, sh, st, x, xm, last, out, k, drop, groups, xo, add, tab); break;
    }
}

void launch_drop_rescale(int logn, const u64 *x, long xs, const u64 *coef, u64 *out, int groups, int kl, int np,
                         const DropAdd &add, const Tables &tab, const Knobs &kn, hipStream_t st, u64 *split_tmp,
                         int cls) {
    if (groups <= 0 || kl <= 0) return;
    const OpDropRescale op{x, xs, coef, out, kl, np, logn, add};
    if (split_tmp) {
        launch_split_fwd(logn, op, split_tmp, groups * kl, tab, st);
        return;
    }
    int prime[kMaxMods];
    drop_primes(kl, prime);
    if (use_loop(groups * kl, prime, kl, tab, kn)) {
        launch_loop<false>(logn, op, prime, kl, groups * kl, tab, st, cls);
        return;
    }
    const int xo = kn.ntt_xcd ? 1 : 0;
    const dim3 grid(xo ? ((groups + 7) / 8) * 8 * kl : groups * kl), blk = ntt_block(logn);
    const size_t sh = ntt_lds(logn);
    switch (logn) {
        case 12: hipLaunchKernelGGL((k_fwd_one<12, OpDropRescale>), grid, blk, sh, st, op, groups * kl, kl, xo, tab); break;
        case 13: hipLaunchKernelGGL((k_fwd_one<13, OpDropRescale>), grid, blk, sh, st, op, groups * kl, kl, xo, tab); break;
        default: hipLaunchKernelGGL((k_fwd_one<14, OpDropRescale>), grid, blk, sh, st, op, groups * kl, kl, xo, tab); break;
    }
}

void launch_drop_rescale_chain(int logn, bool inverse_part, const u64 *x, long xs, u64 *out, int groups, int kl, int np,
                               const DropAdd &add, const Tables &tab, hipStream_t st, u64 *tmp_i, u64 *tmp_f) {
    if (groups <= 0 || kl <= 0) return;
    ResMap im{};                                  // rows kl and P of each polynomial
    im.per = 2;
    im.ngrp = 1;
    im.off = kl;
    im.gstride = xs >> logn;
    im.ostride = xs >> logn;
    im.prime[0] = kl;
    im.prime[1] = np;
    const OpNtt opi{x, im, nullptr, im, logn};
    const OpDropRescale opf{x, xs, nullptr, out, kl, np, logn, add};
    switch (logn) {
        case 12: launch_drop_rescale_chain_one<12>(inverse_part, opi, opf, groups, tmp_i, tmp_f, tab, st); break;
        case 13: launch_drop_rescale_chain_one<13>(inverse_part, opi, opf, groups, tmp_i, tmp_f, tab, st); break;
        default: launch_drop_rescale_chain_one<14>(inverse_part, opi, opf, groups, tmp_i, tmp_f, tab, st); break;
    }
}

void launch_fold_last(int logn, u64 *x, long xs, int groups, int kl, int np, const DropAdd &add, const Tables &tab,
                      hipStream_t st) {
    if (groups <= 0 || !add.mask) return;
    const dim3 grid((1u << logn) / 256, groups), blk(256);
    hipLaunchKernelGGL(k_fold_last, grid, blk, 0, st, x, xs, kl, np, add, logn, tab);
}

void launch_int_ntt(int logn, const int64_t *src, u64 *out, int groups, const PrimeList &pl,
                    const Tables &tab, hipStream_t st) {
    if (groups <= 0) return;
    const dim3 grid(groups * pl.n), blk = ntt_block(logn);
    const size_t sh = ntt_lds(logn);
    switch (logn) {
        case 12: hipLaunchKernelGGL(k_int_ntt<12>, grid, blk, sh, st, src, out, pl, tab); break;
        case 13: hipLaunchKernelGGL(k_int_ntt<13>, grid, blk, sh, st, src, out, pl, tab); break;
        default: hipLaunchKernelGGL(k_int_ntt<14>, grid, blk, sh, st, src, out, pl, tab); break;
    }
}

void keyip_rows(int k, int nq, const Tables &tab, const Knobs &kn, RowSet (&rows)[KIP_CLASSES]) {
    for (RowSet &r : rows) r.n = 0;
    for (int t = 0; t <= k; ++t) {
        const int pt = t < k ? t : nq;
        const int cls = tab.host_fp[pt] ? KIP_FP : (kn.mac_limb && tab.host_lt60[pt]) ? KIP_LIMB : KIP_WIDE;
        rows[cls].t[rows[cls].n++] = t;
    }
}

void launch_keyip(int logn, int k, int cls, const RowSet &rows, const u64 *digits, long db, long dr,
                  const KeyList &keys, int R, u64 *out, long ob, const KeyFold &fold, int B, int nq,
                  const Tables &tab, const Knobs &kn, hipStream_t st) {
    if (R <= 0 || B <= 0 || rows.n <= 0 || cls < 0 || cls >= KIP_CLASSES) return;
    const int pairs = rows.n << (logn - 8);
    const int xo = kn.keyip_xcd ? 1 : 0;
    // kn.keyip_rr rotations per workgroup share each digit word when the digits are hoisted
    // (dr = 0) and the fold term, if any, is the same for every rotation (sr = 0)
    int rr = kn.keyip_rr < 1 ? 1 : kn.keyip_rr > 8 ? 8 : kn.keyip_rr;
    // register budget: a thread holds RR k key words per polynomial (2 VGPRs each, FP64 or 30-bit
    // limb pairs). Sharing each digit word among more rotations wins over occupancy: FP64 rows take
    // RR = 8 at 2 waves per SIMD up to k = 6 (no spill; 8% faster than 4 at 3 waves), else the
    // spill-free 3-wave cap; limb rows RR = 4 up to k = 6 (2 waves, 2 VGPRs spilled; 9% faster than
    // 2 at 3 waves) and 3 at k = 7, 1 at k = 8; 128-bit rows the spill-free 3-wave cap.
    const int words = cls == KIP_FP ? (k <= 6 ? 48 : 28) : cls == KIP_LIMB ? (k <= 7 ? 24 : 12) : 10;
    const int cap = words / k < 1 ? 1 : words / k;
    if (rr > cap) rr = cap;
    if (cls != KIP_FP && rr > 4) rr = 4;          // 6 and 8 rotations only for FP64 rows
    if (rr == 5 || rr == 7) rr -= 1;              // instantiated: 1, 2, 3, 4, 6, 8
    if (dr != 0 || (fold.src && fold.sr != 0)) rr = 1;
    // a workgroup loops over the batch, so a small batch leaves each one little work: up to 4
    // ciphertexts, 2 rotations per workgroup (4x the workgroups of 8) shortened the whole forward
    // pass by 0.6-1.3%; from 8 ciphertexts on, sharing the digit words wins
    if (B <= 4 && rr > 2) rr = 2;
    if (rr > R) rr = R;
    const int RG = (R + rr - 1) / rr;
    const dim3 grid((unsigned)(xo ? ((pairs + 7) / 8) * 8 * RG : pairs * RG)), blk(256);
#define CTL_KIP_ONE(KERNEL, K, RR) \
    hipLaunchKernelGGL((KERNEL<K, RR>), grid, blk, 0, st, digits, db, dr, keys, out, ob, fold, rows, B, R, nq, logn, xo, tab.pc)
#define CTL_KIP_RR(KERNEL, K)                        \
    switch (rr) {                                    \
        case 1: CTL_KIP_ONE(KERNEL, K, 1); break;    \
        case 2: CTL_KIP_ONE(KERNEL, K, 2); break;    \
        case 3: CTL_KIP_ONE(KERNEL, K, 3); break;    \
        default: CTL_KIP_ONE(KERNEL, K, 4); break;   \
    }
#define CTL_KIP_RR8(KERNEL, K)                       \
    switch (rr) {                                    \
        case 6: CTL_KIP_ONE(KERNEL, K, 6); break;    \
        case 8: CTL_KIP_ONE(KERNEL, K, 8); break;    \
        default: CTL_KIP_RR(KERNEL, K)               \
    }
#define CTL_KIP(K)                                                  \
    case K:                                                         \
        if (cls == KIP_FP) { CTL_KIP_RR8(k_keyip_fp, K) }           \
        else if (cls == KIP_LIMB) { CTL_KIP_RR(k_keyip_limb, K) }   \
        else { CTL_KIP_RR(k_keyip, K) }                             \
        break;
    switch (k) {
        CTL_KIP(1) CTL_KIP(2) CTL_KIP(3) CTL_KIP(4) CTL_KIP(5) CTL_KIP(6) CTL_KIP(7) CTL_KIP(8)
        default: break;
    }
#undef CTL_KIP
#undef CTL_KIP_RR8
#undef CTL_KIP_RR
#undef CTL_KIP_ONE
}

// Largest supported giant-step chunk that divides t2 and does not exceed cap.
static int mac_chunk(int t2, int cap) {
    static const int opts[] = {16, 12, 8, 6, 4, 3, 2, 1};   // wider chunks spill registers
    for (int c : opts)
        if (c <= cap && t2 % c == 0) return c;
    return 1;
}

void launch_mac(int logn, const u64 *ct, long ct_sb, const u64 *rot, long rot_sb, const u64 *bank, u64 *inner,
                int B, int rows, int ext_nq, int t1, int t2, const Tables &tab, const Knobs &kn, hipStream_t st,
                int part) {
    // ciphertexts per workgroup: up to 16 for the FP64 kernel (1024 threads), 8 for the integer ones
    const int cts = kn.mac_cts < 1 ? 1 : kn.mac_cts > 16 ? 16 : kn.mac_cts;
    const int by = B < cts ? B : cts, by_int = by < 8 ? by : 8;
    PrimeList all{}, fp{}, in{};
    for (int i = 0; i < rows; ++i) {
        const int pi = (ext_nq >= 0 && i == rows - 1) ? ext_nq : i;
        PrimeList &l = tab.host_fp[pi] ? fp : in;
        l.idx[l.n] = all.idx[all.n] = i;
        l.prime[l.n++] = all.prime[all.n++] = pi;
    }
    const int kc = mac_chunk(t2, kn.mac_chunk_cap);
    if (B <= kn.mac_direct_max) {
        const int kd = mac_chunk(t2, 4);        // few accumulators: more workgroups for one ciphertext
        const dim3 grid((1u << logn) / 64, rows, B * (t2 / kd)), blk(64);
        switch (kd) {
#define CTL_MACD(KD) case KD: hipLaunchKernelGGL(k_mac_direct<KD>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, all, tab.pc); break;
            CTL_MACD(4) CTL_MACD(3) CTL_MACD(2)
            default: hipLaunchKernelGGL(k_mac_direct<1>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, all, tab.pc); break;
#undef CTL_MACD
        }
        return;
    }
    if (fp.n && part != 2) {
        const int kf = mac_chunk(t2, kn.mac_chunk_cap < 12 ? kn.mac_chunk_cap : 12);   // 16 would spill
        const dim3 grid((1u << logn) / 64, fp.n, ((B + by - 1) / by) * (t2 / kf)), blk(64, by);
        switch (kf) {
#define CTL_MAC(KC) case KC: hipLaunchKernelGGL(k_mac_fp<KC>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, fp, tab.pc); break;
            CTL_MAC(12) CTL_MAC(8) CTL_MAC(6) CTL_MAC(4) CTL_MAC(3) CTL_MAC(2)
            default: hipLaunchKernelGGL(k_mac_fp<1>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, fp, tab.pc); break;
#undef CTL_MAC
        }
    }
    if (in.n && part != 1) {
        bool limb = kn.mac_limb != 0;
        for (int y = 0; y < in.n; ++y) limb = limb && tab.host_lt60[in.prime[y]];
        if (limb) {
            // 12 VGPRs per chunk entry; at most 8 (KC = 12 fits at 2 waves per SIMD but runs slower)
            const int kl = mac_chunk(t2, kn.mac_chunk_cap < 8 ? kn.mac_chunk_cap : 8);
            // the kernel interleaves chunks with tiles in blocks of 8 tiles (N / 64 is a multiple of 8)
            const dim3 grid(((1u << logn) / 64) * (t2 / kl), in.n, (B + by_int - 1) / by_int), blk(64, by_int);
            switch (kl) {
#define CTL_MAC(KC) case KC: hipLaunchKernelGGL(k_mac_limb<KC>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, in, tab.pc); break;
                CTL_MAC(8) CTL_MAC(6) CTL_MAC(4) CTL_MAC(3) CTL_MAC(2)
                default: hipLaunchKernelGGL(k_mac_limb<1>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, in, tab.pc); break;
#undef CTL_MAC
            }
            return;
        }
        const dim3 grid((1u << logn) / 64, in.n, ((B + by_int - 1) / by_int) * (t2 / kc)), blk(64, by_int);
        switch (kc) {
#define CTL_MAC(KC) case KC: hipLaunchKernelGGL(k_mac<KC>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, in, tab.pc); break;
            CTL_MAC(16) CTL_MAC(12) CTL_MAC(8) CTL_MAC(6) CTL_MAC(4) CTL_MAC(3) CTL_MAC(2)
            default: hipLaunchKernelGGL(k_mac<1>, grid, blk, 0, st, ct, ct_sb, rot, rot_sb, bank, inner, B, rows, t1, t2, logn, in, tab.pc); break;
#undef CTL_MAC
        }
    }
}

void launch_times_p(int logn, const u64 *in, u64 *out, long o_sb, int B, int k, int nq, const Tables &tab,
                    hipStream_t st) {
    const dim3 grid((1u << logn) / 256, 2 * (k + 1), B), blk(256);
    hipLaunchKernelGGL(k_times_p, grid, blk, 0, st, in, out, o_sb, k, nq, logn, tab.pc, tab.cross);
}

void launch_add_terms(int logn, const u64 *a, long a_sb, const u64 *terms, long t_sb, long t_ss, int S,
                      u64 *out, int B, int k, const Tables &tab, hipStream_t st) {
    const dim3 grid((unsigned)((2L * k << logn) / 256), B), blk(256);
    hipLaunchKernelGGL(k_add_terms, grid, blk, 0, st, a, a_sb, terms, t_sb, t_ss, S, out, k, logn, tab.pc);
}

void launch_sum_gather(int logn, u64 *out, long o_sb, const u64 *base, long ba_sb, const u64 *src, long s_sb,
                       long s_sr, int R, int kk, bool ext, int mask, const GalList &gal, int B, int nq,
                       const Tables &tab, hipStream_t st) {
    const dim3 grid((1u << logn) / 256, 2 * kk, B), blk(256);
    hipLaunchKernelGGL(k_sum_gather, grid, blk, 0, st, out, o_sb, base, ba_sb, src, s_sb, s_sr, R, kk, (int)ext,
                       mask, gal, nq, logn, tab.pc);
}

void launch_tensor(int logn, const u64 *a, const u64 *b, u64 *out, int B, int k, const Tables &tab, hipStream_t st) {
    const dim3 grid((unsigned)(((long)k << logn) / 256), B), blk(256);
    hipLaunchKernelGGL(k_tensor, grid, blk, 0, st, a, b, out, k, logn, tab.pc);
}

void launch_affine(int logn, const u64 *in, u64 *out, int B, int k_in, int k_out, const AffineConst &ac,
                   const Tables &tab, hipStream_t st) {
    const dim3 grid((unsigned)((2L * k_out << logn) / 256), B), blk(256);
    hipLaunchKernelGGL(k_affine, grid, blk, 0, st, in, out, k_in, k_out, ac, logn, tab.pc);
}

void launch_ksk_body(int logn, u64 *key, const u64 *e, const u64 *s, u64 g, int nq, const Tables &tab,
                     hipStream_t st) {
    const dim3 grid((1u << logn) / 256, nq + 1, nq), blk(256);
    hipLaunchKernelGGL(k_ksk_body, grid, blk, 0, st, key, e, s, g, nq, logn, tab.pc, tab.cross);
}

void launch_pk_body(int logn, u64 *pk, const u64 *e, const u64 *s, int nq, const Tables &tab, hipStream_t st) {
    const dim3 grid((1u << logn) / 256, nq), blk(256);
    hipLaunchKernelGGL(k_pk_body, grid, blk, 0, st, pk, e, s, nq, logn, tab.pc);
}

void launch_encrypt(int logn, const u64 *pk, const u64 *in, u64 *ct, int nq, const Tables &tab, hipStream_t st) {
    const dim3 grid((1u << logn) / 256, nq), blk(256);
    hipLaunchKernelGGL(k_encrypt, grid, blk, 0, st, pk, in, ct, nq, logn, tab.pc);
}

void launch_dec_mul(int logn, const u64 *ct, const u64 *s, u64 *out, int k, const Tables &tab, hipStream_t st) {
    const dim3 grid((1u << logn) / 256, k), blk(256);
    hipLaunchKernelGGL(k_dec_mul, grid, blk, 0, st, ct, s, out, k, logn, tab.pc);
}

}  // namespace ctl
