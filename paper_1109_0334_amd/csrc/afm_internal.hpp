// afm_internal.hpp -- shared declarations of the libafm sources (plan, kernel constants,
// non-dimensional force laws, launch helpers).
//
// Non-dimensional form used by every kernel: lengths in nm, time tau = wd t, so one drive period
// is 2 pi and one RK4 step is h = 2 pi / N.  With x_i = q_i / 1 nm the modal equations of the
// paper (Eq. 2 with zeta_i = 1/(2 Q_i), tip-normalised modes) become
//   x_i'' = -Om_i^2 x_i - (Om_i / Q_i) x_i' + G F(d, d') / (k 1 nm) + gamma_i a_nm sin(tau),
// Om_i = w_i / wd, G = (w_0 / wd)^2, d = z_c + sum x_i in nm.  The force law returns the whole
// G F / (k 1 nm) term, so each law folds G, k and the unit conversions into per-trajectory
// constants once (in FP64) before the time loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <functional>
#include <type_traits>
#include <vector>

#include "afm.h"

namespace afm {

constexpr int kMaxModes = AFM_MAX_MODES;
constexpr int kMaxParams = AFM_MAX_PARAMS;
constexpr int kMaxSteps = 4096;  // steps per drive period

// Constants shared by every forward launch of a plan; passed by value as a kernel argument so
// that they sit in scalar registers.
// zero entries after the drive table's 2N + 1, read (never used) by the time loop's prefetch
constexpr int kDrivePad = 8;

struct KConst {
    int32_t nm;            // modes
    int32_t law;           // AFM_LAW_*
    int32_t N;             // steps per period
    int32_t n_cycles;      // default periods per trajectory
    int32_t lockin;        // lock-in periods
    int32_t n_free;        // free parameters
    int32_t drive_mode;    // AFM_DRIVE_*
    int32_t free_index[kMaxParams];
    double params[kMaxParams];  // full SI parameter vector (free slots overwritten per lane)
    double k;              // first-mode stiffness, N/m
    double wd;             // drive angular frequency, rad/s
    double fref;           // drive frequency, Hz (the time unit of a parameter-driven base)
    double steady_rtol;    // > 0: adaptive steady-state exit (stroboscopic point test)
    double G;              // (w0 / wd)^2
    double h;              // 2 pi / N
    double div_nm;         // divergence threshold on |u|, nm
    double dmax;           // largest |drive term| of the table, nm (kFmBlock's bound)
    double om2[kMaxModes];    // (w_i / wd)^2
    double cdamp[kMaxModes];  // w_i / (wd Q_i)
    double gain[kMaxModes];   // gamma_i
    double y0[2 * kMaxModes]; // initial (x_i, x_i') in nm
    const float *drive_f;     // [2N + 1 + kDrivePad] g a_nm sin(pi j / N), FP32 (g = gamma_1
                              // for a point mass, else 1); the last kDrivePad entries are zero
    const double *drive_d;    // [2N + 1 + kDrivePad] same, FP64
    const double *lock_c;     // [N + 1] cos(2 pi p / N), entry N = entry 0
    const double *lock_s;     // [N + 1] sin(2 pi p / N)
};

// ------------------------------------------------------------------------------------------
// precision-specific primitives: FP32 uses the hardware approximations (v_rcp_f32,
// v_sqrt_f32, v_log_f32, v_exp_f32, about 1 ulp); FP64 uses the correctly rounded operations.

template <typename R> struct Ops;
template <> struct Ops<float> {
    __device__ static inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static inline float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static inline float log2(float x) { return __builtin_amdgcn_logf(x); }
    __device__ static inline float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
    __device__ static inline float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    __device__ static inline float max(float a, float b) { return __builtin_fmaxf(a, b); }
    __device__ static inline float abs(float a) { return __builtin_fabsf(a); }
};
template <> struct Ops<double> {
    __device__ static inline double rcp(double x) { return 1.0 / x; }
    __device__ static inline double sqrt(double x) { return ::sqrt(x); }
    __device__ static inline double log2(double x) { return ::log2(x); }
    __device__ static inline double exp2(double x) { return ::exp2(x); }
    __device__ static inline double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    __device__ static inline double max(double a, double b) { return __builtin_fmax(a, b); }
    __device__ static inline double abs(double a) { return __builtin_fabs(a); }
};

// 10^-4.5: sqrt(1 nm) in sqrt(m), used by the Hertz and Kelvin-Voigt terms.
constexpr double kSqrtNano = 3.1622776601683794e-05;

// ------------------------------------------------------------------------------------------
// Force laws.  Each holds its per-trajectory constants in R; add<FM>(d, dd, b) returns
// b + G F / (k 1 nm) for gap d (nm) and gap rate dd (nm per unit tau), written so that the
// addition folds into the law's last multiply.  FM selects how a law with a contact branch is
// evaluated:
//   kFmBranch  per-lane branch, each lane evaluates only its own piece (fewest transcendental
//              ops; the divergent control flow costs scalar instructions, which other waves
//              hide when many share a SIMD)
//   kFmFree    branch-free, both pieces with clamped arguments (no control flow)
//   kFmSkip    the far-field piece always, the contact piece only when some lane of the wave
//              is in contact, behind one wave-uniform branch (fewest issue slots when one wave
//              owns a SIMD and contact is rare); laws without this form treat it as kFmFree
//   kFmFar     the far-field piece only: valid only where no lane can be in contact (the
//              contact piece would add an exact zero), see kFmBlock
//   kFmBlock   for the time loop (forward_impl.hpp integrate): before each block of four RK4
//              steps, one wave-uniform test of a bound on how far every lane's gap can fall
//              within the block; a wave far from contact runs the block as kFmFar, otherwise
//              as kFmFree.  Both add the same terms, so the bits are kFmFree's.  Laws without
//              a block bound (and every per-step loop) treat it as kFmFree
constexpr int kFmBranch = 0;
constexpr int kFmFree = 1;
constexpr int kFmSkip = 2;
constexpr int kFmFar = 3;
constexpr int kFmBlock = 4;

// Bound used by kFmBlock for a point mass: over a block of four steps of size h, every RK4 stage
// state lies within 4h of the block's start in time, and every stage velocity within 4h A of the
// start's, where A bounds |acceleration| = |-om2 (g - z_c) - cd v + F + D| at any stage state.
// Out of contact (gap >= dskip) |F| <= fmax = |BH| / dskip^2 and |D| <= dmax; |g - z_c| and |v|
// can grow within the block by at most 4h (|v0| + 4h A) and 4h A, so
//   A <= (om2 |u0| + (4h om2 + cd) |v0| + fmax + dmax) / (1 - 16 h^2 om2 - 4h cd) = A*.
// Every stage gap is g0 plus a combination with positive weights, summing to at most 4h, of
// stage velocities, each at least v0 - 4h A*; so no stage gap falls below
// g0 - 4h max(0, 4h A* - v0) (v0 the signed gap rate: a tip moving away from the sample can only
// come back by decelerating).  If that is above dskip for every lane of the wave, the whole
// block stays out of contact (the first stage to enter contact would need a larger excursion
// than the bound allows while all earlier stages were out of contact).  The factors carry a few
// percent of margin and the reach an absolute 1e-3 nm, far above FP32 rounding of the stage
// arithmetic.
template <typename R>
struct BlockBound {
    R c_u, c_v, c_f, c_0;  // A* = c_u |u0| + c_v |v0| + c_f fmax + c_0
    R h4, h16;             // reach = h4 max(0, h16 A* - v0) + 1e-3 nm
};

template <int LAW, typename R> struct Law;

// whether a law has the kFmBlock bound (a `kBlock` member that is true)
template <class L, class = void> struct HasBlock : std::false_type {};
template <class L>
struct HasBlock<L, std::void_t<decltype(L::kBlock)>> : std::integral_constant<bool, L::kBlock> {};

// DMT: out of contact BH / d^2 with BH = -G H R / (6 k) (nm^3); in contact the attraction is
// frozen at its d = a0 value and BE (a0 - d)^{3/2} is added, BE = G (4/3) E* sqrt(R) 10^-4.5 / k.
// Branch-free: BH / max(d, a0)^2 + BE max(a0 - d, 0)^{3/2} is the same function.
//
// FP32 form of the Hertz term: with ce = sgn(BE) |BE|^{2/3} and q = ce (a0 - d) clamped to the
// side of zero that ce's sign allows (a median against 0 and +-inf), BE max(a0 - d, 0)^{3/2} =
// q sqrt(|q|).  That is one fma and one median where the plain form needs a subtraction, a
// maximum and a multiplication (the sign handling keeps E* < 0 exact, as the oracle computes it).
template <typename R> struct Law<AFM_LAW_DMT, R> {
    static constexpr bool kRate = false;
    static constexpr bool kBranch = true;
    R zc, a0, BH, BHa, BE, ce, cea0, clim, dskip, fmax;
    Law() = default;
    __device__ Law(const double *p, const KConst &K) {
        const double a0n = p[3] * 1e9;
        // the skip form's contact test d < dskip: the Hertz term of the branch-free form can be
        // nonzero only below ce a0 / ce (FP32-rounded), which lies within a few ulps of a0, so
        // a0 + 2^-20 |a0| is above it; gaps between the two add exact zeros either way
        dskip = (R)(a0n + ::fabs(a0n) * 0x1p-20);
        const double bh = -K.G * p[1] * p[4] / (6.0 * K.k) * 1e27;
        const double be = K.G * (4.0 / 3.0) * p[2] * ::sqrt(p[4]) * kSqrtNano / K.k;
        zc = (R)(p[0] * 1e9);
        a0 = (R)a0n;
        BH = (R)bh;
        BHa = (R)(bh / (a0n * a0n));
        BE = (R)be;
        const double c = be < 0.0 ? -::cbrt(be * be) : ::cbrt(be * be);
        ce = (R)c;
        cea0 = (R)(c * a0n);
        clim = be < 0.0 ? -(R)INFINITY : (R)INFINITY;
        // largest out-of-contact attraction |BH| / d^2 (d >= dskip), rounded up; infinite for a
        // separation at or below zero (the block bound then never skips)
        const double ds = (double)dskip;
        fmax = ds > 0.0 ? (R)(::fabs(bh) / (ds * ds) * (1.0 + 1e-6)) : (R)INFINITY;
    }
    // kFmBlock: whether the gap g (rate v) may come within dskip during the next four steps
    // (see BlockBound); NaN states count as near
    static constexpr bool kBlock = true;
    // ordering key of the small-batch kernel's lanes: trajectories with similar contact
    // stiffness E* sqrt(R) tap at similar phases, so a wave of them is near contact in fewer
    // four-step blocks (any order gives the same results)
    __host__ __device__ static double contact_key(const double *p) {
        return p[2] * ::sqrt(::fabs(p[4]));
    }
    __device__ inline bool near(R g, R v, const BlockBound<R> &bb) const {
        const R av = Ops<R>::abs(v);
        const R Am = Ops<R>::fma(bb.c_u, Ops<R>::abs(g - zc),
                                 Ops<R>::fma(bb.c_v, av, Ops<R>::fma(bb.c_f, fmax, bb.c_0)));
        const R reach = Ops<R>::fma(bb.h4, Ops<R>::max(Ops<R>::fma(bb.h16, Am, -v), R(0)), R(1e-3));
        return !(g - reach > dskip);
    }
    template <int FM> __device__ inline R add(R d, R, R b) const {
        if constexpr (std::is_same<R, float>::value) {
            if constexpr (FM == kFmFar) {
                // only used where every stage gap is at least dskip > a0 (the block bound), so
                // max(d, a0) = d and this is the branch-free form's far-field piece bit for bit
                const R r = Ops<R>::rcp(d);
                return Ops<R>::fma(BH * r, r, b);
            } else if constexpr (FM != kFmBranch) {
                // max(d, a0) as a median against the largest finite float (equal for every
                // finite d): IEEE-mode v_max would first quiet both operands, two extra
                // instructions per pass of the time loop
                const R r = Ops<R>::rcp(__builtin_amdgcn_fmed3f(d, a0, R(3.4028234663852886e38)));
                R f = Ops<R>::fma(BH * r, r, b);
                // the Hertz term is zero unless d < a0 (up to the rounding of ce a0); the skip
                // form skips it only when every lane of the wave is above dskip, where the
                // branch-free form adds an exact zero, so both give the same bits in every lane
                if (FM != kFmSkip || __builtin_amdgcn_ballot_w64(d < dskip) != 0) {
                    // a scheduling barrier (no instruction, no memory effect) keeps the compiler
                    // from speculating this block into a select evaluated on every pass
                    if constexpr (FM == kFmSkip) __builtin_amdgcn_sched_barrier(0);
                    const R q = __builtin_amdgcn_fmed3f(Ops<R>::fma(-ce, d, cea0), R(0), clim);
                    f = Ops<R>::fma(q, Ops<R>::sqrt(__builtin_fabsf(q)), f);
                }
                return f;
            } else {
                R f;
                if (d > a0) {
                    const R r = Ops<R>::rcp(d);
                    f = Ops<R>::fma(BH * r, r, b);
                } else {
                    const R q = Ops<R>::fma(-ce, d, cea0);
                    f = Ops<R>::fma(q, Ops<R>::sqrt(__builtin_fabsf(q)), b + BHa);
                }
                return f;
            }
        } else {
            if constexpr (FM == kFmFar) {
                const R r = Ops<R>::rcp(d);  // d >= dskip > a0 (see the FP32 form)
                return Ops<R>::fma(BH * r, r, b);
            } else if constexpr (FM != kFmBranch) {
                const R r = Ops<R>::rcp(Ops<R>::max(d, a0));
                const R del = Ops<R>::max(a0 - d, R(0));
                return Ops<R>::fma(BE * del, Ops<R>::sqrt(del), Ops<R>::fma(BH * r, r, b));
            } else {
                R f;
                if (d > a0) {
                    const R r = Ops<R>::rcp(d);
                    f = Ops<R>::fma(BH * r, r, b);
                } else {
                    const R del = a0 - d;
                    f = Ops<R>::fma(BE * del, Ops<R>::sqrt(del), b + BHa);
                }
                return f;
            }
        }
    }

    // Gradient support: F and its partials with respect to d, d' and the constants
    // c = (BH, BE, a0); to_si() maps accumulated dJ/dc and dJ/dz_c to SI parameter derivatives.
    static constexpr int NC = 3;
    __device__ inline R grad(R d, R, R &Fd, R &Fdd, R (&dc)[NC]) const {
        const bool out = d > a0;
        const R m = out ? d : a0;
        const R r = Ops<R>::rcp(m);
        const R del = out ? R(0) : a0 - d;
        const R s = Ops<R>::sqrt(del);
        const R r3 = BH * r * r * r;
        Fd = out ? R(-2) * r3 : R(-1.5) * BE * s;
        Fdd = R(0);
        dc[0] = r * r;
        dc[1] = del * s;
        dc[2] = out ? R(0) : R(-2) * r3 + R(1.5) * BE * s;
        return Ops<R>::fma(BH * r, r, BE * del * s);
    }
    __device__ static void to_si(const double *p, const KConst &K, const double (&sc)[NC],
                                 double szc, double *g) {
        const double bh = -K.G * p[1] * p[4] / (6.0 * K.k) * 1e27;
        const double be = K.G * (4.0 / 3.0) * p[2] * ::sqrt(p[4]) * kSqrtNano / K.k;
        g[0] = szc * 1e9;
        g[1] = sc[0] * bh / p[1];
        g[2] = sc[1] * be / p[2];
        g[3] = sc[2] * 1e9;
        g[4] = sc[0] * bh / p[4] + sc[1] * be / (2.0 * p[4]);
    }
};

// Lennard-Jones type: BL / d [(r0/d)^n - (r0/d)^m], BL = G eps n m / (n - m) / (k 1e-18).
// Each term as one power of two: (r0/d)^n / d = exp2(n log2 r0 - (n + 1) log2 d), so the
// force takes one log2, two exp2 and no reciprocal; d <= 0 gives NaN.
template <typename R> struct Law<AFM_LAW_LJ, R> {
    static constexpr bool kRate = false;
    static constexpr bool kBranch = false;
    R zc, BL, lr0, n, m, nl, ml, n1, m1;
    Law() = default;
    __device__ Law(const double *p, const KConst &K) {
        const double l = ::log2(p[2] * 1e9);
        zc = (R)(p[0] * 1e9);
        BL = (R)(K.G * p[1] * p[3] * p[4] / (p[3] - p[4]) / (K.k * 1e-18));
        lr0 = (R)l;
        n = (R)p[3];
        m = (R)p[4];
        nl = (R)(p[3] * l);
        ml = (R)(p[4] * l);
        n1 = (R)(-(p[3] + 1.0));
        m1 = (R)(-(p[4] + 1.0));
    }
    template <int FM> __device__ inline R add(R d, R, R b) const {
        const R ld = Ops<R>::log2(d);
        return Ops<R>::fma(BL, Ops<R>::exp2(Ops<R>::fma(n1, ld, nl)) -
                                   Ops<R>::exp2(Ops<R>::fma(m1, ld, ml)), b);
    }

    // constants c = (BL, lr0, n, m)
    static constexpr int NC = 4;
    __device__ inline R grad(R d, R, R &Fd, R &Fdd, R (&dc)[NC]) const {
        const R r = Ops<R>::rcp(d);
        const R ls = lr0 - Ops<R>::log2(d);
        const R En = Ops<R>::exp2(n * ls), Em = Ops<R>::exp2(m * ls);
        const R ln2 = R(0.69314718055994531);
        const R Br = BL * r;
        Fd = -Br * r * ((n + R(1)) * En - (m + R(1)) * Em);
        Fdd = R(0);
        dc[0] = r * (En - Em);
        dc[1] = Br * ln2 * (n * En - m * Em);
        dc[2] = Br * ln2 * ls * En;
        dc[3] = -Br * ln2 * ls * Em;
        return Br * (En - Em);
    }
    __device__ static void to_si(const double *p, const KConst &K, const double (&sc)[NC],
                                 double szc, double *g) {
        const double eps = p[1], r0 = p[2], n_ = p[3], m_ = p[4];
        const double bl = K.G * eps * n_ * m_ / (n_ - m_) / (K.k * 1e-18);
        g[0] = szc * 1e9;
        g[1] = sc[0] * bl / eps;
        g[2] = sc[1] / (r0 * 0.69314718055994531);
        g[3] = sc[2] + sc[0] * bl * (-m_ / (n_ * (n_ - m_)));
        g[4] = sc[3] + sc[0] * bl * (n_ / (m_ * (n_ - m_)));
    }
};

// Kelvin-Voigt contact: DMT plus BV sqrt(a0 - d) d' in contact, BV = -G eta wd sqrt(R)
// 10^-4.5 / k (the viscous force -eta sqrt(R delta) d' with d' = wd 1 nm x').
template <typename R> struct Law<AFM_LAW_KV, R> {
    static constexpr bool kRate = true;
    static constexpr bool kBranch = true;
    // FP32 form of the contact piece as for DMT: with q = ce (a0 - d) clamped by a median
    // (ce = sgn(BE) |BE|^{2/3}, |ce| >= 1e-30 so that E* = 0 stays finite), the Hertz and
    // viscous terms are sqrt(|q|) (q + BVs d') with BVs = BV / sqrt(|ce|).
    R zc, a0, BH, BHa, BE, BV, ce, cea0, clim, BVs, dskip, fmax;
    Law() = default;
    __device__ Law(const double *p, const KConst &K) {
        const double a0n = p[3] * 1e9;
        const double bh = -K.G * p[1] * p[4] / (6.0 * K.k) * 1e27;
        const double be = K.G * (4.0 / 3.0) * p[2] * ::sqrt(p[4]) * kSqrtNano / K.k;
        const double bv = -K.G * p[5] * K.wd * ::sqrt(p[4]) * kSqrtNano / K.k;
        zc = (R)(p[0] * 1e9);
        a0 = (R)a0n;
        BH = (R)bh;
        BHa = (R)(bh / (a0n * a0n));
        BE = (R)be;
        BV = (R)bv;
        const double m = ::fmax(::cbrt(be * be), 1e-30);
        const double c = be < 0.0 ? -m : m;
        ce = (R)c;
        cea0 = (R)(c * a0n);
        clim = be < 0.0 ? -(R)INFINITY : (R)INFINITY;
        BVs = (R)(bv / ::sqrt(m));
        // the block test's threshold and largest out-of-contact attraction, as for DMT (the
        // viscous term, like the Hertz term, vanishes with q)
        dskip = (R)(a0n + ::fabs(a0n) * 0x1p-20);
        const double ds = (double)dskip;
        fmax = ds > 0.0 ? (R)(::fabs(bh) / (ds * ds) * (1.0 + 1e-6)) : (R)INFINITY;
    }
    // kFmBlock: out of contact the law is DMT's far field, so DMT's block bound holds
    static constexpr bool kBlock = true;
    __host__ __device__ static double contact_key(const double *p) {
        return p[2] * ::sqrt(::fabs(p[4]));
    }
    __device__ inline bool near(R g, R v, const BlockBound<R> &bb) const {
        const R av = Ops<R>::abs(v);
        const R Am = Ops<R>::fma(bb.c_u, Ops<R>::abs(g - zc),
                                 Ops<R>::fma(bb.c_v, av, Ops<R>::fma(bb.c_f, fmax, bb.c_0)));
        const R reach = Ops<R>::fma(bb.h4, Ops<R>::max(Ops<R>::fma(bb.h16, Am, -v), R(0)), R(1e-3));
        return !(g - reach > dskip);
    }
    template <int FM> __device__ inline R add(R d, R dd, R b) const {
        if constexpr (FM == kFmFar) {
            // only where every stage gap is at least dskip > a0 (the block bound): q = 0 there,
            // and the branch-free form adds sqrt(0) (q + BVs d') = an exact zero
            const R r = Ops<R>::rcp(d);
            return Ops<R>::fma(BH * r, r, b);
        } else if constexpr (std::is_same<R, float>::value) {
            if constexpr (FM != kFmBranch) {
                const R r = Ops<R>::rcp(__builtin_amdgcn_fmed3f(d, a0, R(3.4028234663852886e38)));
                const R q = __builtin_amdgcn_fmed3f(Ops<R>::fma(-ce, d, cea0), R(0), clim);
                return Ops<R>::fma(Ops<R>::sqrt(__builtin_fabsf(q)), Ops<R>::fma(BVs, dd, q),
                                   Ops<R>::fma(BH * r, r, b));
            } else {
                R f;
                if (d > a0) {
                    const R r = Ops<R>::rcp(d);
                    f = Ops<R>::fma(BH * r, r, b);
                } else {
                    const R q = Ops<R>::fma(-ce, d, cea0);
                    f = Ops<R>::fma(Ops<R>::sqrt(__builtin_fabsf(q)), Ops<R>::fma(BVs, dd, q),
                                    b + BHa);
                }
                return f;
            }
        } else {
            if constexpr (FM != kFmBranch) {
                const R r = Ops<R>::rcp(Ops<R>::max(d, a0));
                const R del = Ops<R>::max(a0 - d, R(0));
                return Ops<R>::fma(Ops<R>::sqrt(del), Ops<R>::fma(BE, del, BV * dd),
                                   Ops<R>::fma(BH * r, r, b));
            } else {
                R f;
                if (d > a0) {
                    const R r = Ops<R>::rcp(d);
                    f = Ops<R>::fma(BH * r, r, b);
                } else {
                    const R del = a0 - d;
                    const R s = Ops<R>::sqrt(del);
                    f = Ops<R>::fma(s, Ops<R>::fma(BE, del, BV * dd), b + BHa);
                }
                return f;
            }
        }
    }

    // constants c = (BH, BE, BV, a0)
    static constexpr int NC = 4;
    __device__ inline R grad(R d, R dd, R &Fd, R &Fdd, R (&dc)[NC]) const {
        const bool out = d > a0;
        const R m = out ? d : a0;
        const R r = Ops<R>::rcp(m);
        const R del = out ? R(0) : a0 - d;
        const R s = Ops<R>::sqrt(del);
        const R r3 = BH * r * r * r;
        // d sqrt(delta)/d delta = 1/(2 sqrt(delta)), taken as 0 on the contact boundary
        const R hs = s > R(0) ? R(0.5) * BV * dd * Ops<R>::rcp(s) : R(0);
        Fd = out ? R(-2) * r3 : R(-1.5) * BE * s - hs;
        Fdd = BV * s;
        dc[0] = r * r;
        dc[1] = del * s;
        dc[2] = s * dd;
        dc[3] = out ? R(0) : R(-2) * r3 + R(1.5) * BE * s + hs;
        return Ops<R>::fma(BH * r, r, s * (BE * del + BV * dd));
    }
    __device__ static void to_si(const double *p, const KConst &K, const double (&sc)[NC],
                                 double szc, double *g) {
        const double bh = -K.G * p[1] * p[4] / (6.0 * K.k) * 1e27;
        const double be = K.G * (4.0 / 3.0) * p[2] * ::sqrt(p[4]) * kSqrtNano / K.k;
        const double bv = -K.G * p[5] * K.wd * ::sqrt(p[4]) * kSqrtNano / K.k;
        g[0] = szc * 1e9;
        g[1] = sc[0] * bh / p[1];
        g[2] = sc[1] * be / p[2];
        g[3] = sc[3] * 1e9;
        g[4] = sc[0] * bh / p[4] + sc[1] * be / (2.0 * p[4]) + sc[2] * bv / (2.0 * p[4]);
        g[5] = sc[2] * bv / p[5];
    }
};

// Hooke (Eq. 3): BK d for d < 0, BK = -G k_s / k.
template <typename R> struct Law<AFM_LAW_HOOKE, R> {
    static constexpr bool kRate = false;
    static constexpr bool kBranch = false;
    R zc, BK;
    Law() = default;
    __device__ Law(const double *p, const KConst &K) {
        zc = (R)(p[0] * 1e9);
        BK = (R)(-K.G * p[1] / K.k);
    }
    template <int FM> __device__ inline R add(R d, R, R b) const {
        return d < R(0) ? Ops<R>::fma(BK, d, b) : b;
    }

    static constexpr int NC = 1;
    __device__ inline R grad(R d, R, R &Fd, R &Fdd, R (&dc)[NC]) const {
        const bool in = d < R(0);
        Fd = in ? BK : R(0);
        Fdd = R(0);
        dc[0] = in ? d : R(0);
        return in ? BK * d : R(0);
    }
    __device__ static void to_si(const double *p, const KConst &K, const double (&sc)[NC],
                                 double szc, double *g) {
        g[0] = szc * 1e9;
        g[1] = sc[0] * (-K.G / K.k);
    }
};

// Spring-damper (Eq. 4): BK d + BS d' for d < 0, BS = -G zeta_s wd / k.
template <typename R> struct Law<AFM_LAW_SD, R> {
    static constexpr bool kRate = true;
    static constexpr bool kBranch = false;
    R zc, BK, BS;
    Law() = default;
    __device__ Law(const double *p, const KConst &K) {
        zc = (R)(p[0] * 1e9);
        BK = (R)(-K.G * p[1] / K.k);
        BS = (R)(-K.G * p[2] * K.wd / K.k);
    }
    template <int FM> __device__ inline R add(R d, R dd, R b) const {
        return d < R(0) ? Ops<R>::fma(BK, d, Ops<R>::fma(BS, dd, b)) : b;
    }

    static constexpr int NC = 2;
    __device__ inline R grad(R d, R dd, R &Fd, R &Fdd, R (&dc)[NC]) const {
        const bool in = d < R(0);
        Fd = in ? BK : R(0);
        Fdd = in ? BS : R(0);
        dc[0] = in ? d : R(0);
        dc[1] = in ? dd : R(0);
        return in ? BK * d + BS * dd : R(0);
    }
    __device__ static void to_si(const double *p, const KConst &K, const double (&sc)[NC],
                                 double szc, double *g) {
        g[0] = szc * 1e9;
        g[1] = sc[0] * (-K.G / K.k);
        g[2] = sc[1] * (-K.G * K.wd / K.k);
    }
};

template <typename R> struct Law<AFM_LAW_NONE, R> {
    static constexpr bool kRate = false;
    static constexpr bool kBranch = false;
    R zc;
    Law() = default;
    __device__ Law(const double *p, const KConst &) { zc = (R)(p[0] * 1e9); }
    template <int FM> __device__ inline R add(R, R, R b) const { return b; }

    static constexpr int NC = 1;  // no constants; one unused slot keeps array types valid
    __device__ inline R grad(R, R, R &Fd, R &Fdd, R (&dc)[NC]) const {
        Fd = R(0);
        Fdd = R(0);
        dc[0] = R(0);
        return R(0);
    }
    __device__ static void to_si(const double *, const KConst &, const double (&)[NC], double szc,
                                 double *g) {
        g[0] = szc * 1e9;
    }
};

// ------------------------------------------------------------------------------------------
// Forward launch description (device pointers; see afm_forward_batch / afm_misfit).
struct FwdArgs {
    int64_t n;                 // trajectories
    int64_t ld;                // leading dimension of theta ([n_free][ld])
    const double *theta;
    const int32_t *n_cycles;   // per trajectory (or per group, see group) or NULL
    const int32_t *target_id;  // per trajectory or NULL
    const double *targets;     // [n_targets][W] or NULL
    int32_t n_targets;
    int32_t group;             // > 0: n_cycles and target_id are indexed by i / group
    int32_t row_by_group;      // without target_id: target row = i / group (else row 0)
    double *amp, *phase, *J, *trace;
    int32_t *status;
    const double *base;        // optional per-group full parameter vectors [kMaxParams][base_ld]
    int64_t base_ld;           // (indexed by i / group, or i when group == 0)
    const int32_t *items;      // persistent queue: item order (NULL = plain grid launch)
    int32_t n_items, chunks;   // items = groups x chunks of 64 lanes
    int32_t *head;             // queue head counter (reset to 0 before the launch)
    double *mtrace;            // optional window modal coordinates, m: [NM][W][mtrace_ld]
    int64_t mtrace_ld;         // (trajectory fastest)
    int32_t *periods;          // optional periods integrated per trajectory
    int32_t xcd_stride;        // plain k_forward grid: > 1 = only every xcd_stride-th workgroup works
    const int32_t *order;      // plain k_forward: lane slot -> trajectory (NULL = identity)
    int32_t *order_buf;        // plan-owned [kOrderMax] buffers the launcher may use to build
    double *key_buf;           // `order` (NULL = do not reorder)
};

// Adjoint launch description (see afm_grad_batch).
struct GradArgs {
    int64_t n, ld;
    const double *theta;
    const int32_t *n_cycles;
    const int32_t *target_id;
    const double *targets;
    int32_t n_targets;
    int32_t group;
    double *J, *dJ;        // J [n], dJ [n_free][ld]
    int32_t *status;
    float *ckpt;           // [segments][4 NM][n] (FP64 plans: doubles)
    float *seg;            // [kc][2 NM + 1][n]
    int32_t kc;            // checkpoint stride in RK4 steps
    const double *base;    // optional per-point full parameter vectors [kMaxParams][base_ld]
    int64_t base_ld;
    int32_t mp;            // mode-parallel kernel (one lane per mode; several modes only)
    int32_t form;          // kGradSweep or kGradSegments (see grad.hip)
};

// Forms of the adjoint: one reverse sweep per trajectory, or every checkpoint segment
// differentiated on its own lane (tangent columns) and the segments combined afterwards.
constexpr int32_t kGradSweep = 1;
constexpr int32_t kGradSegments = 2;

// ------------------------------------------------------------------------------------------
// host side

struct GraphCache;

}  // namespace afm

namespace afm {
// Launch shape of a plain forward launch and the plan's record of tuned shapes.
struct FwdShape {
    int32_t block;  // lanes per workgroup: 64, 128 or 256
    int32_t tpl;    // trajectories per lane: 1 or 2; 0 = mode-parallel (one lane per mode)
};
struct FwdTune {
    int64_t n;       // batch size
    int32_t prec;    // AFM_PREC_*
    int32_t has_nc;  // per-trajectory period counts given
    FwdShape shape;
    float ms;        // the winning candidate's time
};
}  // namespace afm

struct afm_plan {
    afm_problem prob;
    int32_t precision;
    int32_t device;
    afm::KConst kc;
    float *d_drive_f = nullptr;
    double *d_drive_d = nullptr;
    double *d_lock = nullptr;       // [2 (N + 1)]
    int32_t *d_order = nullptr;     // [kOrderMax] lane order of small forward batches
    double *d_order_keys = nullptr; // [kOrderMax] their keys
    hipStream_t stream = nullptr;   // private stream used to capture and replay graphs
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // plan-owned workspace for afm_invert
    void *ws = nullptr;
    size_t ws_bytes = 0;
    afm::GraphCache *graph = nullptr;
    int32_t n_cu = 0;               // compute units of the plan's device (persistent grids)
    // plan-owned workspace for afm_grad_batch and the tuned checkpoint stride per batch size
    void *gws = nullptr;
    size_t gws_bytes = 0;
    int64_t tuned_n = -1;
    int32_t tuned_kc = 0;
    int32_t tuned_mp = 0;
    int32_t tuned_form = 0;
    int32_t grad_form = 0;          // afm_set_grad_form: 0 = automatic, else a pinned form
    // plan-owned workspace for afm_polish
    void *pws = nullptr;
    size_t pws_bytes = 0;
    // plan-owned workspace for afm_forward_points (window modal coordinates)
    void *mws = nullptr;
    size_t mws_bytes = 0;
    // plan-owned work-queue order of afm_misfit_swarms and the inputs it was built for
    void *qws = nullptr;
    size_t qws_bytes = 0;
    const int32_t *q_ncyc = nullptr;
    int32_t q_S = 0, q_P = 0;
    // PSO constants
    double pso_w, pso_c1, pso_c2, pso_vmax;
    // tuned launch shapes of plain forward launches (filled on first use of a batch size)
    mutable std::vector<afm::FwdTune> fwd_tune;
    afm::FwdShape pinned_shape{0, 0};  // block 0: tuned
};

namespace afm {

// thread-local error text
void set_error(const std::string &msg);
afm_status fail(afm_status code, const std::string &msg);
afm_status hip_fail(hipError_t e, const char *what);

// full parameter vector of lane/point `g`: the plan's fixed values or a per-group override,
// with the free parameters written in from theta (column i)
__device__ inline void load_params(double (&p)[kMaxParams], const KConst &K, const double *base,
                                   int64_t base_ld, int64_t g, const double *theta, int64_t ld,
                                   int64_t i) {
#pragma unroll
    for (int q = 0; q < kMaxParams; ++q) {
        p[q] = base ? base[q * base_ld + g] : K.params[q];
#pragma unroll
        for (int j = 0; j < kMaxParams; ++j)
            if (j < K.n_free && K.free_index[j] == q) p[q] = theta[(int64_t)j * ld + i];
    }
}

// launchers (forward.hip, pso.hip)
hipError_t launch_forward(const afm_plan *plan, const FwdArgs &a, hipStream_t s);
hipError_t launch_swarm_init(const afm_plan *plan, const afm_swarm &sw, uint64_t seed,
                             hipStream_t s);
hipError_t launch_pso_step(const afm_plan *plan, const afm_swarm &sw, const double *J,
                           uint64_t seed, int32_t iter, int32_t is_last, double cutoff,
                           hipStream_t s);
hipError_t launch_gather_best(const afm_plan *plan, const afm_swarm &sw, double *best_theta,
                              double *best_J, int32_t *gen, hipStream_t s);

// precision-explicit variants take AFM_PREC_*; the plain ones use the plan's precision
hipError_t launch_grad(const afm_plan *plan, const GradArgs &a, hipStream_t s);
hipError_t launch_grad_p(const afm_plan *plan, int32_t prec, const GradArgs &a, hipStream_t s);
hipError_t launch_forward_p(const afm_plan *plan, int32_t prec, const FwdArgs &a, hipStream_t s);
// Batches at and above this many trajectories are treated as GPU-filling (256-lane workgroups,
// the force-law forms of throughput-bound launches); below it one wave owns a SIMD.
constexpr int64_t kSmallBatch = 65536;
// largest small batch whose lanes are ordered by the law's contact key (see launch_plain)
constexpr int64_t kOrderMax = 16384;
// the forward kernels of one force law and precision (forward_impl.hpp, instantiated by the
// forward_<law>_<precision>.hip units)
template <int LAW, bool MIXED>
hipError_t launch_fwd_law(const afm_plan *plan, const FwdArgs &a, const KConst &K, hipStream_t s);
// whether the plan already holds a (tuned or pinned) shape for this plain forward launch
bool forward_shape_known(const afm_plan *plan, int32_t prec, const FwdArgs &a);
// tuned (or, under stream capture, default) shape of a plain forward launch; `launch` runs one
// candidate on the real arguments
hipError_t forward_shape(const afm_plan *plan, int32_t prec, const FwdArgs &a, int nm,
                         hipStream_t s, const std::function<hipError_t(FwdShape)> &launch,
                         FwdShape *out);
size_t grad_ckpt_bytes(const afm_plan *plan, int32_t prec, int64_t n, int32_t kc);
// segment buffer (kGradSweep) or segment records (kGradSegments) of a gradient launch
size_t grad_seg_bytes(const afm_plan *plan, int32_t prec, int64_t n, int32_t kc, int32_t form);
// whether the segment-parallel form is built for the plan's problem
bool grad_segments_ok(const afm_plan *plan);
// the form a gradient launch takes when no tuning applies: the pinned form, else the segment
// form where it is built, else the sweep
int32_t grad_default_form(const afm_plan *plan);
int32_t polish_prec(const afm_plan *plan);

// L-BFGS polish (lbfgs.hip)
size_t polish_total_bytes(const afm_plan *plan, int64_t n, int32_t kc);
hipError_t enqueue_polish(afm_plan *plan, void *ws, int64_t n, double *z,
                          const int32_t *target_id, const double *targets, int32_t n_targets,
                          const int32_t *n_cycles, const double *base, int32_t steps, int32_t kc,
                          double *J_out, hipStream_t s);
hipError_t enqueue_topk(const afm_plan *plan, const afm_swarm &sw, int32_t k, int32_t *taken,
                        double *zsel, int32_t *tsel, const int32_t *ncyc, int32_t *nsel,
                        const double *swarm_base, double *bsel, hipStream_t s);
hipError_t enqueue_merge(const afm_swarm &sw, int32_t k, const double *zsel, const double *Jsel,
                         hipStream_t s);
constexpr int32_t kPolishStride = 64;  // checkpoint stride of the polish's gradients

// argument checks shared by the entry points
afm_status check_forward_args(const afm_plan *plan, int64_t n, const double *theta);

}  // namespace afm
