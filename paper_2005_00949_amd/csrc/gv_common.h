// gv_common.h -- device-side constants, precision policies and counter-based
// random numbers of the gfx950 stepping library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gv {

// CODATA 2018 constants (MeV, cm)
constexpr double kMe = 0.51099895;
constexpr double kRe = 2.8179403262e-13;
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kNA = 6.02214076e23;
constexpr double kKB = 2.99792458;          // p[MeV] = kKB * B[T] * R[cm]
constexpr double kPi = 3.14159265358979323846;
constexpr double kInf = 1.0e300;

// particle types; queue index == type
enum : int { kGamma = 0, kElectron = 1, kPositron = 2 };
// step limiters
enum : int { kLimPhys = 0, kLimEloss = 1, kLimGeom = 2, kLimField = 3 };
// processes (interaction counters)
enum : int { kCompton = 0, kPair = 1, kMoller = 2, kBhabha = 3, kBremsEm = 4, kBremsEp = 5,
             kAnnih = 6, kNull = 7, kNProc = 8 };
// random-stream purposes: low 8 bits of the fourth counter word
enum : uint32_t { kPurpStep = 0, kPurpMsc = 1, kPurpChild = 2, kPurpAnnih = 3, kPurpFs0 = 16,
                  kFsMaxIter = 240 };
// track status after a step (kParked: stopped at its RK45 move, waiting in
// the batched driver's integration queue)
enum : int { kAlive = 0, kDead = 1, kEscaped = 2, kKilled = 3, kParked = 4 };
// per-material table record columns (4 per node and particle type)
//   gamma: Sigma_compton, Sigma_pair, -, -
//   e-   : Sigma_moller, Sigma_brems, S (restricted dE/dx), R (range)
//   e+   : Sigma_bhabha, Sigma_brems, S, R
constexpr int kCols = 4;
constexpr int kOutside = -1;

// ---------------------------------------------------------------------------
// Precision policies.  P64: everything in double.  PMix: sampling, tables,
// direction and kinetic energy in float; position, boundary distances, safety
// and deposit accumulation in double.
// ---------------------------------------------------------------------------
struct P64 {
    using R = double;
    static constexpr bool kMixed = false;
};
struct PMix {
    using R = float;
    static constexpr bool kMixed = true;
};

// Overloaded device math so that stage code is written once per policy.  The
// double versions are the accurate library functions; the float versions use
// the gfx950 hardware transcendentals (log2/exp2/sin/cos units, a few ulp),
// which keep every single-step output within its 1e-5 budget.  Sine and
// cosine are the exception on |x| <= pi/4: the hardware units have an
// absolute error near 5e-7 there, i.e. a large relative error for the small
// angles that dominate (scattering angles, pair opening angles, the helix
// phase of one step), and those errors decorrelate mixed-precision histories
// from their FP64 twins; there the Taylor polynomials through x^9 and x^10
// (truncation below 3e-9 relative at pi/4) are used instead.

__device__ __forceinline__ float sin_small(float x)
{
    const float x2 = x * x;
    return x * (1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f + x2 * (-1.0f / 5040.0f + x2 * (1.0f / 362880.0f)))));
}
__device__ __forceinline__ float cos_small(float x)
{
    const float x2 = x * x;
    return 1.0f + x2 * (-0.5f + x2 * (1.0f / 24.0f + x2 * (-1.0f / 720.0f + x2 * (1.0f / 40320.0f +
                                                                                   x2 * (-1.0f / 3628800.0f)))));
}
constexpr float kQuarterPi = 0.78539816f;
__device__ __forceinline__ double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_log(float x) { return __logf(x); }
__device__ __forceinline__ double m_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float m_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_exp(float x) { return __expf(x); }
__device__ __forceinline__ double m_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float m_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sin(double x) { return sin(x); }
__device__ __forceinline__ float m_sin(float x) { return fabsf(x) <= kQuarterPi ? sin_small(x) : __sinf(x); }
__device__ __forceinline__ double m_cos(double x) { return cos(x); }
__device__ __forceinline__ float m_cos(float x) { return fabsf(x) <= kQuarterPi ? cos_small(x) : __cosf(x); }
__device__ __forceinline__ double m_atan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ float m_atan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double m_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float m_pow(float x, float y) { return __powf(x, y); }
__device__ __forceinline__ double m_log10(double x) { return log10(x); }
__device__ __forceinline__ float m_log10(float x) { return __log10f(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float m_min(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double m_max(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float m_max(float a, float b) { return fmaxf(a, b); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw; SC'11): ten rounds of two 32x32
// multiplies with a half swap, key bumped by the golden-ratio Weyl constants.
// Every track draws blocks keyed by the run seed at counter
// (event, track id lo, track id hi, step << 8 | purpose): one independent
// stream per track, as in the per-track pseudo-random trees of Sec. 5.1.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t w[4];
};

__host__ __device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * c0;
        const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    U4 o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

__device__ __forceinline__ U4 stream_block(uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep,
                                           uint32_t purpose)
{
    return philox(event, (uint32_t)tid, (uint32_t)(tid >> 32), ((nstep & 0xFFFFFFu) << 8) | purpose,
                  (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in (0, 1] from two words (first = high), exact in double;
// the float version is the double value rounded once.
__device__ __forceinline__ double u53_d(uint32_t a, uint32_t b)
{
    const uint64_t x = ((((uint64_t)a) << 32) | b) >> 11;
    return (double)(x + 1) * 0x1p-53;
}
// 32-bit uniform in (0, 1]
__device__ __forceinline__ double u32_d(uint32_t w) { return ((double)w + 1.0) * 0x1p-32; }

template <class R> __device__ __forceinline__ R u53(uint32_t a, uint32_t b) { return (R)u53_d(a, b); }
template <class R> __device__ __forceinline__ R u32(uint32_t w) { return (R)u32_d(w); }

// Exponential variate with full relative precision at both ends: -log(u) for
// u <= 1/2, -log1p(-v) with v = 1 - u formed exactly from the integer
// complement for u > 1/2.
template <class R> __device__ __forceinline__ R expo(uint32_t a, uint32_t b)
{
    const uint64_t x = ((((uint64_t)a) << 32) | b) >> 11;
    if (x < (1ull << 52)) return -m_log((R)((double)(x + 1) * 0x1p-53));
    const R v = (R)((double)((1ull << 53) - 1ull - x) * 0x1p-53);
    return -m_log1p(-v);
}

}  // namespace gv
