// lbm_device.h -- device-side data layout and per-node arithmetic of the
// IFDLBM step (arXiv:2306.07603), shared by the fused and staged kernels.
//
// State of a node: the nine deviations g_k = f-hat_k - omega_k rho0 of the
// distribution f-hat (Eq. 2.3) and the relaxation time lambda that produced
// them (Eq. 2.14).  Working with deviations drops rho0 from every formula
// (the collision, the difference stencils and the boundary extrapolation are
// affine with weights summing to one, or linear with weights summing to
// zero) and keeps FP32 rounding on the O(u, P) part only.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ifd {

enum Precision { P_FP64 = 0, P_FP32 = 1, P_FP16DEV = 2, P_FP32X = 3, P_FP32SR = 4, P_FP32SRF = 5 };

// ------------------------------------------------------- random bits
// Integer mixing function (the "lowbias32" finaliser of C. Wellons's hash
// prospector): a bijection of 32-bit words with good avalanche.
__host__ __device__ inline uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Random words of one node at one step, a function of (step key, cavity,
// node index) only, so that every kernel and every work decomposition draws
// the same bits: h = mix32(step_key ^ cav_key ^ node), then four xorshift32
// steps (Marsaglia's 13/17/5 triple) give five words; population k uses the
// 16 bits r16(k) of word k / 2.
__host__ __device__ inline uint32_t cavity_key(int cav) { return mix32((uint32_t)cav * 0x9E3779B9u + 0x632BE5ABu); }
__host__ __device__ inline uint32_t step_key(uint32_t counter, uint32_t step) { return mix32(counter ^ mix32(step + 0x85EBCA6Bu)); }

struct NodeWords {
    uint32_t w[5];
    __device__ __forceinline__ NodeWords(uint32_t skey, uint32_t ckey, uint32_t node)
    {
        uint32_t x = mix32(skey ^ ckey ^ node);
        x = x ? x : 0x6D2B79F5u;   // xorshift32 has no zero state
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            w[m] = x;
            x ^= x << 13;
            x ^= x >> 17;
            x ^= x << 5;
        }
    }
    __device__ __forceinline__ uint32_t r16(int k) const { return k & 1 ? w[k >> 1] >> 16 : w[k >> 1] & 0xFFFFu; }
};

// Stochastic rounding of an FP64 value to FP32: add 16 random bits at the top
// of the 29 significand bits that FP32 drops, then truncate them.  The result
// is the FP32 neighbour above (in magnitude) with probability equal to the
// dropped fraction rounded down to a multiple of 2^-16, so the rounding error
// has zero mean up to 2^-16 ulp; the truncated value converts to FP32 exactly
// (normal range).
__device__ __forceinline__ float round_stochastic(double v, uint32_t r16)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    b += (unsigned long long)r16 << 13;
    b &= ~0x1FFFFFFFull;
    return (float)__longlong_as_double((long long)b);
}

// One cavity in the device tables.  Planes are SoA: population k of node
// (i, j) lives at f_off + k * plane + j * pitch + i.
struct CavityDesc {
    int32_t nx, ny, pitch, active;
    int64_t f_off;      // element offset of plane 0 in the distribution arrays
    int64_t plane;      // elements per plane (ny * pitch)
    int64_t l_off;      // element offset in the lambda arrays
    int64_t geo_off;    // a_j at geo_off + j (ny entries), s_i at geo_off + ny + i (nx entries)
    double dt;          // time step
    double K;           // consistency coefficient, Eq. (2.15.1)
    double expo;        // (n - 1) / 2, the exponent of Eq. (1.4) on gamma^2
    double g2min;       // gamma_min^2
    double mix;         // central weight of Eq. (2.5)
    double u_lid;       // lid velocity, Eq. (1.5)
    double inv2dxi;     // 1 / (2 dxi)
    double inv2deta;    // 1 / (2 deta)
    double lam_newton;  // K / c_s^2, lambda of the Newtonian case
    double lam0;        // initial lambda, U L / (Re c_s^2)
    double cot;         // 1 / tan(theta), exactly 0 at 90 degrees
    double dxi, deta;   // grid spacings of the computational square
    int32_t newtonian;  // n == 1 exactly
    int32_t index;      // cavity index in the handle
    int32_t implicit_lambda;   // Step (2) solved for its own fixed point instead of lagged
};

// ---------------------------------------------------------------- storage
// F: stored distribution element; L: stored lambda; T: arithmetic of the
// distributions; V: arithmetic of Step (2) and of the relaxation coefficients
// (a function of the state, not a stored increment, so FP32 there perturbs the
// viscosity by O(1e-7) relative and shifts no fixed point).  cvt / enc convert
// between F and T (enc rounds to nearest).

template <int PREC> struct Storage;

template <> struct Storage<P_FP64> {
    static constexpr bool kStochastic = false;
    static constexpr bool kExactFinal = false;
    using F = double;
    using L = double;
    using T = double;
    using V = double;
    __device__ static inline T cvt(F v, int) { return v; }
    __device__ static inline F enc(T v, int) { return v; }
    __device__ static inline T load(const F* p, int64_t i, int k) { return cvt(p[i], k); }
    __device__ static inline void store(F* p, int64_t i, int k, T v) { p[i] = enc(v, k); }
};

template <> struct Storage<P_FP32> {
    static constexpr bool kStochastic = false;
    static constexpr bool kExactFinal = false;
    using F = float;
    using L = float;
    using T = float;
    using V = float;
    __device__ static inline T cvt(F v, int) { return v; }
    __device__ static inline F enc(T v, int) { return v; }
    __device__ static inline T load(const F* p, int64_t i, int k) { return cvt(p[i], k); }
    __device__ static inline void store(F* p, int64_t i, int k, T v) { p[i] = enc(v, k); }
};

// FP32 storage with FP64 arithmetic: only the stored state is rounded to FP32.
template <> struct Storage<P_FP32X> {
    static constexpr bool kStochastic = false;
    static constexpr bool kExactFinal = false;
    using F = float;
    using L = float;
    using T = double;
    using V = double;
    __device__ static inline T cvt(F v, int) { return (T)v; }
    __device__ static inline F enc(T v, int) { return (F)v; }
    __device__ static inline T load(const F* p, int64_t i, int k) { return cvt(p[i], k); }
    __device__ static inline void store(F* p, int64_t i, int k, T v) { p[i] = enc(v, k); }
};

// FP32 storage, FP64 arithmetic of the distributions, distributions stored
// with stochastic rounding: at a steady state the rounding of the stored
// state no longer acts as a constant forcing (with round-to-nearest it
// shifts, and can freeze, the fixed point).
template <> struct Storage<P_FP32SR> {
    static constexpr bool kStochastic = true;
    static constexpr bool kExactFinal = false;
    using F = float;
    using L = float;
    using T = double;
    using V = float;
    __device__ static inline T cvt(F v, int) { return (T)v; }
    __device__ static inline F enc(T v, int) { return (F)v; }
    __device__ static inline F enc_sr(T v, int, uint32_t r16) { return round_stochastic(v, r16); }
    __device__ static inline T load(const F* p, int64_t i, int k) { return cvt(p[i], k); }
    __device__ static inline void store(F* p, int64_t i, int k, T v) { p[i] = enc(v, k); }
};

// FP32 storage with stochastic rounding, FP32 arithmetic, except where the
// exact stored g meets a small increment: e - g of Step (2) is formed in FP64,
// and the new value g + (collision increment of Eq. 2.15 + streaming increment
// of Eq. 3.6) is summed in FP64 from the stored g and rounded stochastically
// (the increments are FP32, each accurate relative to itself; the staged
// schedule rebuilds f-hat+ in FP64 instead).  The rounding errors left in FP32
// are those of increments and of the half-step values that only enter
// difference stencils, not of a stored state.
template <> struct Storage<P_FP32SRF> {
    static constexpr bool kStochastic = true;
    static constexpr bool kExactFinal = true;
    using F = float;
    using L = float;
    using T = float;
    using V = float;
    __device__ static inline T cvt(F v, int) { return v; }
    __device__ static inline F enc(T v, int) { return v; }
    __device__ static inline F enc_sr(double v, int, uint32_t r16) { return round_stochastic(v, r16); }
    __device__ static inline T load(const F* p, int64_t i, int k) { return cvt(p[i], k); }
    __device__ static inline void store(F* p, int64_t i, int k, T v) { p[i] = enc(v, k); }
};

// Encoding of a new state population: stochastic rounding where the storage asks for it.
template <typename S, typename X>
__device__ __forceinline__ typename S::F encode_state(X v, int k, const NodeWords* nw)
{
    if constexpr (S::kStochastic)
        return S::enc_sr(v, k, nw->r16(k));
    else
        return S::enc(v, k);
}

// FP16 storage of g_k / omega_k: the division by the lattice weight puts all
// nine planes on the same O(3 P + 3 c.u) scale, inside FP16's normal range.
// New states are rounded stochastically: on fine grids the change of a
// population per step is far below an FP16 ulp (2^-11 relative), and round to
// nearest would drop it every step.
template <> struct Storage<P_FP16DEV> {
    static constexpr bool kStochastic = true;
    static constexpr bool kExactFinal = false;
    using F = __half;
    using L = float;
    using T = float;
    using V = float;
    __device__ static inline float w(int k) { return k == 0 ? 4.0f / 9.0f : (k < 5 ? 1.0f / 9.0f : 1.0f / 36.0f); }
    __device__ static inline float inv_w(int k) { return k == 0 ? 2.25f : (k < 5 ? 9.0f : 36.0f); }
    __device__ static inline T cvt(F v, int k) { return w(k) * __half2float(v); }
    __device__ static inline F enc(T v, int k) { return __float2half_rn(v * inv_w(k)); }
    // The 13 significand bits of the FP32 value below FP16's are added to 13
    // random bits and dropped: the kept value rounds up with probability equal
    // to the dropped fraction.  Below FP16's normal range (|x| < 2^-14) the
    // final conversion rounds to nearest on the subnormal grid.
    __device__ static inline F enc_sr(T v, int k, uint32_t r16)
    {
        const float x = v * inv_w(k);
        const uint32_t b = __float_as_uint(x);
        if ((b & 0x7F800000u) == 0x7F800000u) return __float2half_rn(x);   // inf, nan
        return __float2half_rn(__uint_as_float((b + (r16 >> 3)) & ~0x1FFFu));
    }
    __device__ static inline T load(const F* p, int64_t i, int k) { return cvt(p[i], k); }
    __device__ static inline void store(F* p, int64_t i, int k, T v) { p[i] = enc(v, k); }
};

// ----------------------------------------------------------------- lattice
// Eq. (2.9): c_k = (cx, cy); omega = 4/9, 1/9 (k = 1..4), 1/36 (k = 5..8);
// omegabar_0 = -5/9, omegabar_k = omega_k otherwise; c_s^2 = 1/3.

__host__ __device__ constexpr int cxk(int k) { return k == 1 || k == 5 || k == 8 ? 1 : (k == 3 || k == 6 || k == 7 ? -1 : 0); }
__host__ __device__ constexpr int cyk(int k) { return k == 2 || k == 5 || k == 6 ? 1 : (k == 4 || k == 7 || k == 8 ? -1 : 0); }

// Eqs. (2.10)-(2.11) on deviations: u = sum c_k g_k and
// P = (c_s^2 / omegabar_0) (-sum_{k>0} g_k + omega_0 |u|^2 / (2 c_s^2)) = 0.6 s - 0.4 |u|^2.
template <typename T>
__device__ __forceinline__ void moments(const T g[9], T& P, T& ux, T& uy)
{
    ux = (g[1] - g[3]) + (g[5] - g[6]) - (g[7] - g[8]);
    uy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const T s = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    P = T(0.6) * s - T(0.4) * (ux * ux + uy * uy);
}

// Eq. (2.8) minus omega_k rho0, with the second-order term over 2 c_s^4:
// e_0 = -5/3 P - 2/3 |u|^2, e_k = omega_k (3 P + 3 c.u + 4.5 (c.u)^2 - 1.5 |u|^2).
// In FP64 the velocity term is written with a = 1.5 c.u as 2 a (a + 1) =
// a (2 a + 2): every constant of that form is an inline operand of the FP64
// FMA (3 and 4.5 are not, and VOP3 takes no literal), and c.u of a lattice
// direction is a signed sum of a_x = 1.5 u_x and a_y = 1.5 u_y, so no product
// with a zero velocity component is formed.  equilibrium_k is the same
// arithmetic population by population.
template <typename T>
__device__ __forceinline__ T eq_velocity_term(T cu)   // FP32: 3 c.u + 4.5 (c.u)^2
{
    return cu * (T(3) + T(4.5) * cu);
}
__device__ __forceinline__ double eq_velocity_term_a(double a)   // FP64: a = 1.5 c.u
{
    return a * __builtin_fma(a, 2.0, 2.0);
}

// a = 1.5 c_k.u of population k (FP64) from a_x = 1.5 u_x and a_y = 1.5 u_y
__device__ __forceinline__ double eq_a(int k, double ax, double ay)
{
    switch (k) {
    case 1: return ax;
    case 2: return ay;
    case 3: return -ax;
    case 4: return -ay;
    case 5: return ax + ay;
    case 6: return ay - ax;
    case 7: return -(ax + ay);
    default: return ax - ay;
    }
}

template <typename T>
__device__ __forceinline__ void equilibrium(T P, T ux, T uy, T e[9])
{
    const T uu = ux * ux + uy * uy;
    const T base = T(3) * P - T(1.5) * uu;
    const T w1 = T(1) / T(9), w5 = T(1) / T(36);
    e[0] = T(-5) / T(3) * P - T(2) / T(3) * uu;
    if constexpr (std::is_same<T, double>::value) {
        const double ax = __builtin_fma(0.5, ux, ux), ay = __builtin_fma(0.5, uy, uy);
#pragma unroll
        for (int k = 1; k < 9; ++k) e[k] = (k < 5 ? w1 : w5) * (base + eq_velocity_term_a(eq_a(k, ax, ay)));
    } else {
        auto q = [&](T cu) { return base + eq_velocity_term(cu); };
        e[1] = w1 * q(ux);
        e[2] = w1 * q(uy);
        e[3] = w1 * q(-ux);
        e[4] = w1 * q(-uy);
        e[5] = w5 * q(ux + uy);
        e[6] = w5 * q(uy - ux);
        e[7] = w5 * q(-ux - uy);
        e[8] = w5 * q(ux - uy);
    }
}

// Population k of Eq. (2.8) alone (same arithmetic as equilibrium()).
template <typename T>
__device__ __forceinline__ T equilibrium_k(T P, T ux, T uy, int k)
{
    const T uu = ux * ux + uy * uy;
    const T base = T(3) * P - T(1.5) * uu;
    const T w = k < 5 ? T(1) / T(9) : T(1) / T(36);
    if (k == 0) return T(-5) / T(3) * P - T(2) / T(3) * uu;
    if constexpr (std::is_same<T, double>::value) {
        const double ax = __builtin_fma(0.5, ux, ux), ay = __builtin_fma(0.5, uy, uy);
        return w * (base + eq_velocity_term_a(eq_a(k, ax, ay)));
    } else {
        const T cu = k == 1 ? ux : k == 2 ? uy : k == 3 ? -ux : k == 4 ? -uy
                   : k == 5 ? ux + uy : k == 6 ? uy - ux : k == 7 ? -ux - uy : ux - uy;
        return w * (base + eq_velocity_term(cu));
    }
}

// 1/x for x > 0: v_rcp_f32 (1 ulp) in FP32; v_rcp_f64 refined by two Newton
// steps r <- r (2 - x r) in FP64 (relative error squares at each step).
template <typename T> __device__ __forceinline__ T recip(T x);
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double recip<double>(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = r * __builtin_fma(-x, r, 2.0);
    r = r * __builtin_fma(-x, r, 2.0);
    return r;
}

#ifdef __HIP_DEVICE_COMPILE__
// x^y in FP64 for the power law of Step (2): x = gamma^2 >= gamma_min^2 > 0
// and |y ln x| below 700.  exp(y ln x) from textbook methods, within about
// two ulp (measured against an 80-bit pow over x in [1e-14, 1e8], y in
// [-0.5, 2]), in a fifth of the instructions of the general pow, which also
// handles x <= 0, infinities and integer y:
//  * ln x: x = m 2^k with m in [sqrt(1/2), sqrt(2)), and ln m = 2 atanh(s),
//    s = (m - 1) / (m + 1), |s| <= 0.172, by its Taylor series through s^21
//    (truncation below 1e-17 relative);
//  * z = y ln x as a rounded high part and a low part: ln 2 is split so that
//    k ln2_hi is exact, and the rounding error of y (k ln2_hi) is kept;
//  * exp: the reduction z = n ln 2 + r, |r| <= ln 2 / 2, of Cody and Waite
//    (n ln2_hi exact, ln2_lo applied separately), the Taylor series of e^r
//    through r^13 (truncation below 5e-18 relative), and the scaling by 2^n.
// A NaN x (a diverged state) gives NaN.
__device__ __forceinline__ double pow_pos_f64(double x, double y)
{
    constexpr double kLn2Hi = 0x1.62e42fefa38p-1;     // ln 2 to 42 bits: n ln2_hi is exact for |n| < 2^11
    constexpr double kLn2Lo = 0x1.ef35793c7673p-45;   // ln 2 - kLn2Hi
    constexpr double kLog2e = 0x1.71547652b82fep+0;   // 1 / ln 2
    constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
    int k = __builtin_amdgcn_frexp_exp(x);            // x = m' 2^k, m' in [1/2, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    const bool low = m < kSqrtHalf;                   // m' < sqrt(1/2): m = 2 m', k - 1
    m = low ? m + m : m;
    k = low ? k - 1 : k;
    // s = (m - 1) / (m + 1) to about half an ulp: m - 1 and the rounding error de of d = m + 1 are exact, and one
    // correction step of the quotient takes out the errors of the reciprocal and of d
    const double d = m + 1.0, de = m - (d - 1.0), rd = recip(d), s0 = (m - 1.0) * rd;
    const double s = __builtin_fma(__builtin_fma(-s0, d, m - 1.0) - s0 * de, rd, s0);
    const double s2 = s * s;
    double t = 1.0 / 21.0;                            // (atanh(s) / s - 1) / s^2 = 1/3 + s^2/5 + ... + s^18/21
    t = __builtin_fma(t, s2, 1.0 / 19.0);
    t = __builtin_fma(t, s2, 1.0 / 17.0);
    t = __builtin_fma(t, s2, 1.0 / 15.0);
    t = __builtin_fma(t, s2, 1.0 / 13.0);
    t = __builtin_fma(t, s2, 1.0 / 11.0);
    t = __builtin_fma(t, s2, 1.0 / 9.0);
    t = __builtin_fma(t, s2, 1.0 / 7.0);
    t = __builtin_fma(t, s2, 1.0 / 5.0);
    t = __builtin_fma(t, s2, 1.0 / 3.0);
    const double s_2 = s + s;
    const double lnm = __builtin_fma(s_2 * s2, t, s_2);
    const double kd = (double)k;
    const double lhi = kd * kLn2Hi;                   // exact
    const double llo = __builtin_fma(kd, kLn2Lo, lnm);
    const double zh = y * lhi;
    const double zl = __builtin_fma(y, llo, __builtin_fma(y, lhi, -zh));   // y lhi - zh is exact
    const double n = __builtin_rint((zh + zl) * kLog2e);
    double r = __builtin_fma(-n, kLn2Hi, zh);         // below 1.1 in magnitude, to 2^-53
    r = __builtin_fma(-n, kLn2Lo, r + zl);
    double p = 1.0 / 6227020800.0;                    // 1/13!, then Horner down to 1/0!
    p = __builtin_fma(p, r, 1.0 / 479001600.0);
    p = __builtin_fma(p, r, 1.0 / 39916800.0);
    p = __builtin_fma(p, r, 1.0 / 3628800.0);
    p = __builtin_fma(p, r, 1.0 / 362880.0);
    p = __builtin_fma(p, r, 1.0 / 40320.0);
    p = __builtin_fma(p, r, 1.0 / 5040.0);
    p = __builtin_fma(p, r, 1.0 / 720.0);
    p = __builtin_fma(p, r, 1.0 / 120.0);
    p = __builtin_fma(p, r, 1.0 / 24.0);
    p = __builtin_fma(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)n);
}
#endif

template <typename T> __host__ __device__ __forceinline__ T pow_pos(T x, T y);
template <> __host__ __device__ __forceinline__ double pow_pos<double>(double x, double y)
{
#ifdef __HIP_DEVICE_COMPILE__
    return pow_pos_f64(x, y);
#else
    return pow(x, y);
#endif
}
template <> __host__ __device__ __forceinline__ float pow_pos<float>(float x, float y)
{
    // x >= gamma_min^2 > 0 is a normal float: v_log_f32 / v_exp_f32 (base 2) on the device
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
#else
    return exp2f(y * log2f(x));
#endif
}

// Step (2): lambda from the non-equilibrium second moment, Eqs. (2.12)-(2.14)
// and (1.4).  With f from f-hat by Eq. (2.18), f - f_eq = 2 lam_old (g - e) /
// (2 lam_old + dt), so D = (grad u + grad u^T)/2 = -3 Pi / (2 lam_old + dt)
// with Pi = sum_k c_k c_k (g_k - e_k), and 2 D:D = 18 (Pxx^2 + 2 Pxy^2 + Pyy^2)
// / (2 lam_old + dt)^2.  mu = K max(2 D:D, gamma_min^2)^((n-1)/2), lambda = mu / c_s^2.
// The parameters of Step (2) in the arithmetic type, converted once per work item.
template <typename T>
struct PowerLaw {
    T K3, expo, g2min, dt, lam_newton;
    bool newtonian, implicit;
    __host__ __device__ __forceinline__ explicit PowerLaw(const CavityDesc& c)
        : K3(T(3) * T(c.K)), expo(T(c.expo)), g2min(T(c.g2min)), dt(T(c.dt)), lam_newton(T(c.lam_newton)),
          newtonian(c.newtonian != 0), implicit(c.implicit_lambda != 0)
    {
    }
};

// Implicit Step (2): lambda = K3 max(18 Q / s^2, gamma_min^2)^expo with
// s = 2 lambda + dt, Q = Pi:Pi.  h(lambda) = lambda - map(lambda) is negative
// at 0 and crosses zero once below `hi` (for expo >= 0 the map falls from
// map(0); for expo < 0 it rises, concave in s, up to the floor's value).
// Newton steps h' = 1 + 4 expo map / s from the lagged value, replaced by
// bisection of the bracket whenever a step leaves it or h' <= 0.
template <typename V>
__host__ __device__ __forceinline__ V implicit_relaxation_time(V Q18, V lam0, const PowerLaw<V>& pl)
{
    auto map = [&](V lam, bool& floored) {
        const V s = V(2) * lam + pl.dt;
        V g2 = Q18 / (s * s);
        floored = !(g2 > pl.g2min);
        g2 = floored ? pl.g2min : g2;
        return pl.K3 * pow_pos<V>(g2, pl.expo);
    };
    bool fl;
    V lo = V(0), hi = pl.expo >= V(0) ? map(V(0), fl) : pl.K3 * pow_pos<V>(pl.g2min, pl.expo);
    V lam = lam0 > lo && lam0 < hi ? lam0 : V(0.5) * (lo + hi);
    // Newton converges quadratically: a step below tol leaves an error far below it
    const V tol = sizeof(V) == 8 ? V(1e-13) : V(1e-6);
    for (int it = 0; it < 40; ++it) {
        const V m = map(lam, fl);
        const V h = lam - m;
        if (h == V(0)) break;   // exact root
        if (h < V(0))
            lo = lam;
        else
            hi = lam;
        const V s = V(2) * lam + pl.dt;
        const V hp = V(1) + (fl ? V(0) : V(4) * pl.expo * m / s);
        V next = hp > V(0) ? lam - h / hp : V(-1);
        if (!(next >= lo && next <= hi)) next = V(0.5) * (lo + hi);
        const V step = next > lam ? next - lam : lam - next;
        lam = next;
        if (step <= tol * lam) break;
    }
    return lam;
}

template <typename T>
__device__ __forceinline__ T relaxation_time(const T g[9], const T e[9], T lam_old, const PowerLaw<T>& pl)
{
    if (pl.newtonian) return pl.lam_newton;
    T n[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) n[k] = g[k] - e[k];
    const T s58 = (n[5] + n[6]) + (n[7] + n[8]);
    const T pxx = (n[1] + n[3]) + s58;
    const T pyy = (n[2] + n[4]) + s58;
    const T pxy = (n[5] - n[6]) + (n[7] - n[8]);
    const T r = recip(T(2) * lam_old + pl.dt);
    T gamma2 = T(18) * (pxx * pxx + T(2) * pxy * pxy + pyy * pyy) * r * r;
    gamma2 = gamma2 > pl.g2min ? gamma2 : pl.g2min;
    return pl.K3 * pow_pos<T>(gamma2, pl.expo);
}

template <typename T>
__device__ __forceinline__ T relaxation_time(const T g[9], const T e[9], T lam_old, const CavityDesc& c)
{
    return relaxation_time(g, e, lam_old, PowerLaw<T>(c));
}

// Step (2) in the arithmetic V from d_k = e_k - g_k (T): Pi = -sum c c d, and
// only its quadratic form enters gamma^2, so the sign drops out.  IMPLICIT
// selects the fixed-point form (the cavity's implicit_lambda flag).
template <bool IMPLICIT, typename T, typename V>
__device__ __forceinline__ V relaxation_time_d(const T d[9], V lam_old, const PowerLaw<V>& pl)
{
    if (pl.newtonian) return pl.lam_newton;
    const T s58 = (d[5] + d[6]) + (d[7] + d[8]);
    const V pxx = V((d[1] + d[3]) + s58);
    const V pyy = V((d[2] + d[4]) + s58);
    const V pxy = V((d[5] - d[6]) + (d[7] - d[8]));
    if constexpr (IMPLICIT) return implicit_relaxation_time(V(18) * (pxx * pxx + V(2) * pxy * pxy + pyy * pyy), lam_old, pl);
    const V r = recip(V(2) * lam_old + pl.dt);
    V gamma2 = V(18) * (pxx * pxx + V(2) * pxy * pxy + pyy * pyy) * r * r;
    gamma2 = gamma2 > pl.g2min ? gamma2 : pl.g2min;
    return pl.K3 * pow_pos<V>(gamma2, pl.expo);
}

// Eqs. (2.15)-(2.16) written as x + b (e - x): f-hat+ = g + b_hat (e - g),
// b_hat = 2 dt / (2 lam + dt); f-bar+ = g + b_bar (e - g), b_bar = 3 dt / (4 lam
// + 2 dt).  Rounding of b perturbs the relaxation rate only: mass and
// momentum stay exactly those of g.
template <typename V>
struct Relax {
    V b_hat, b_bar;
    __device__ __forceinline__ Relax(V lam, V dt)
    {
        const V r = recip(V(2) * lam + dt);
        b_hat = V(2) * dt * r;
        b_bar = V(1.5) * dt * r;
    }
};

// Eq. (2.17) as f = f-bar + b (e - f-bar), b = dt / (4 lam + dt).
template <typename V>
__device__ __forceinline__ V half_coef(V lam, V dt)
{
    return dt * recip(V(4) * lam + dt);
}

// Steps (3)-(4): Eq. (2.15) f-hat+ = ((2 lam - dt) g + 2 dt e) / (2 lam + dt) and
// Eq. (2.16) f-bar+ = ((4 lam - dt) g + 3 dt e) / (4 lam + 2 dt).
template <typename T>
struct Collision {
    T a_hat, b_hat, a_bar, b_bar;
    __device__ __forceinline__ Collision(T lam, T dt)
    {
        const T r = recip(T(2) * lam + dt);
        a_hat = (T(2) * lam - dt) * r;
        b_hat = T(2) * dt * r;
        a_bar = (T(4) * lam - dt) * (T(0.5) * r);
        b_bar = T(1.5) * dt * r;
    }
};

// Eq. (2.17): f = (4 lam f-bar + dt e) / (4 lam + dt).
template <typename T>
struct HalfStep {
    T a, b;
    __device__ __forceinline__ HalfStep(T lam, T dt)
    {
        const T r = recip(T(4) * lam + dt);
        a = T(4) * lam * r;
        b = dt * r;
    }
};

// Eq. (2.5) with (2.6)-(2.7): eps * central + (1 - eps) * second-order upwind,
// times 2h, from the five points m2, m1, c0, p1, p2 along one grid line.  The
// upwind side follows the sign of the contravariant velocity (c >= 0: points
// behind).  Where the second upwind point would leave the grid (lo_edge for
// c >= 0, hi_edge for c < 0) the first-order one-sided difference is used.
template <typename T>
__device__ __forceinline__ T mixed_diff_2h(T m2, T m1, T c0, T p1, T p2, bool c_nonneg, bool lo_edge, bool hi_edge, T eps)
{
    const T cen = p1 - m1;
    T up;
    if (c_nonneg)
        up = lo_edge ? T(2) * (c0 - m1) : (T(3) * c0 - T(4) * m1) + m2;
    else
        up = hi_edge ? T(2) * (p1 - c0) : (T(4) * p1 - T(3) * c0) - p2;
    return eps * cen + (T(1) - eps) * up;
}

// Boundary classification and the non-equilibrium extrapolation neighbour
// (one index inward, diagonal at corners).
__device__ __forceinline__ bool is_boundary(int i, int j, int nx, int ny)
{
    return i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
}

__device__ __forceinline__ void inward(int i, int j, int nx, int ny, int& ni, int& nj)
{
    ni = i == 0 ? 1 : (i == nx - 1 ? nx - 2 : i);
    nj = j == 0 ? 1 : (j == ny - 1 ? ny - 2 : j);
}

// Non-equilibrium extrapolation onto a wall node from the nine values x_nb of
// its inward neighbour: x_b = f_eq(P_nb, u_wall) + (x_nb - f_eq(P_nb, u_nb)).
template <typename T>
__device__ __forceinline__ void extrapolate(const T xnb[9], T uwall, T xb[9])
{
    T P, ux, uy, e_nb[9], e_w[9];
    moments(xnb, P, ux, uy);
    equilibrium(P, ux, uy, e_nb);
    equilibrium(P, uwall, T(0), e_w);
#pragma unroll
    for (int k = 0; k < 9; ++k) xb[k] = e_w[k] + (xnb[k] - e_nb[k]);
}

}  // namespace ifd
