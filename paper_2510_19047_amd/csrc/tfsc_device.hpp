// Device math for the semi-coherent time-frequency statistic (gfx950).
//
// * Track: 2PN TaylorT3 in theta = [eta (t_c - t) / (5 M)]^(-1/8), evaluated
//   in FP64 with a fixed sequence of IEEE +, -, *, / and sqrt (this file is
//   compiled with -ffp-contract=off), so the bin index, track end and N_seg
//   are reproducible bit for bit on any IEEE machine.
// * Tranche spectrum: the paper's Fresnel-kernel form, Eq. (fresnel-ft),
//   rewritten exactly in bin-relative variables (see tranche_spectrum_bin).
// * Response: rigid analytic orbits, single-link transfers and equal-arm
//   TDI-1.5 A/E evaluated once per tranche at (t_m, f_m), Eq. (tdi2).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace tfsc {

constexpr double kPi = 3.141592653589793;
constexpr double kTwoPi = 6.283185307179586;
constexpr double kMsunS = 4.925490947e-6;
constexpr double kFdotRef = 1.34e-12;
constexpr double kClight = 299792458.0;
constexpr double kYearS = 31557600.0;
constexpr double kArmM = 2.5e9;
constexpr double kAuM = 1.495978707e11;
constexpr int kHalfBins = 10;  // N_F = 2 * 10 + 1

enum : int { kFlagInvalid = 1, kFlagEmpty = 2, kFlagBandEnd = 4, kFlagMergeEnd = 8, kFlagAllExcluded = 16 };

// ------------------------------------------------------------------ track
struct Track {
    double eta, M, c8, a2, a3, a4, b2, b3, b4, tc, th0;
    double M5, M40;               // 5M and 40M, each rounded once
    double r5M, rc8, r40M, reta;  // correctly rounded 1/(5M), 1/c8, 1/(40M), 1/eta
};

// The correctly rounded quotient a/b from yb = RN(1/b): q = RN(a yb) is within an ulp of a/b,
// the residual a - b q is exact in one FMA, and RN(q + r yb) is RN(a/b) (Markstein's theorem for
// binary floating point with round-to-nearest, no underflow or overflow).  Three FP64
// operations instead of a full division, with the same result bit for bit.
__device__ __forceinline__ double div_rn(double a, double b, double yb) {
    const double q = a * yb;
    const double r = fma(-b, q, a);
    return fma(r, yb, q);
}

// sqrt(x), correctly rounded, for a positive normal x >= 2^-767 (the track's q and its roots): Goldschmidt's
// iteration from the hardware reciprocal square root y ~ 1/sqrt(x) (g -> sqrt(x), h -> 1/(2 sqrt(x))), one
// refinement of both, then two corrections of g by the exact residual x - g^2.  This is the sequence the
// compiler emits for sqrt(double) without its rescaling of tiny inputs and its selects for 0 and infinity,
// so on these inputs it returns the same bits with eight fewer instructions.
__device__ __forceinline__ double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}

// 1/b, correctly rounded, for a normal b whose reciprocal is normal and far from the range limits (the track's
// 1/s and 1/theta^5): the hardware reciprocal refined by two Newton steps, then Markstein's correction of the
// quotient by its exact residual 1 - b q.  This is the compiler's division sequence for 1/b without its operand
// rescaling and its special-value fix-up, so on these inputs it returns the same bits.
__device__ __forceinline__ double rcp_rn(double b) {
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    const double r = fma(-b, y, 1.0);
    return fma(r, y, y);
}

__device__ __forceinline__ bool params_valid(double mc, double eta, double f0, double ct, double ci) {
    if (!(mc > 0.0) || !(eta >= 0.01) || !(eta <= 0.25) || !(f0 > 0.0)) return false;
    if (!(fabs(ct) <= 1.0) || !(fabs(ci) <= 1.0)) return false;
    if (!isfinite(mc) || !isfinite(eta) || !isfinite(f0) || !isfinite(ct) || !isfinite(ci)) return false;
    return true;
}

// Per-template constants: eta^(1/5) by 12 Newton steps from 1, M = Mc eta^(-3/5),
// theta0 with f(theta0) = f0 by a 10-step cube root (from z^(1/4)) and 6 Newton
// steps on the 2PN f(theta), t_c = 5 M theta0^-8 / eta.
__device__ inline void track_init(Track &T, double mc, double eta, double f0) {
    double y = 1.0;
    for (int i = 0; i < 12; ++i) {
        double y4 = (y * y) * (y * y);
        y = (4.0 * y + eta / y4) / 5.0;
    }
    T.eta = eta;
    T.M = (mc * kMsunS) / ((y * y) * y);
    double e2 = eta * eta;
    T.a2 = 743.0 / 2688.0 + (11.0 / 32.0) * eta;
    T.a3 = -3.0 * kPi / 10.0;
    T.a4 = (1855099.0 / 14450688.0 + (56975.0 / 258048.0) * eta) + (371.0 / 2048.0) * e2;
    T.b2 = 3715.0 / 8064.0 + (55.0 / 96.0) * eta;
    T.b3 = -3.0 * kPi / 4.0;
    T.b4 = (9275495.0 / 14450688.0 + (284875.0 / 258048.0) * eta) + (1855.0 / 2048.0) * e2;
    T.c8 = (8.0 * kPi) * T.M;
    double z = T.c8 * f0;
    double r = sqrt(sqrt(z));
    for (int i = 0; i < 10; ++i) r = (2.0 * r + z / (r * r)) / 3.0;
    double th = r;
    for (int i = 0; i < 6; ++i) {
        double th2 = th * th, th3 = th2 * th, th4 = th2 * th2;
        double P = ((1.0 + T.a2 * th2) + T.a3 * th3) + T.a4 * th4;
        double F = th3 * P - z;
        double dP = ((3.0 + (5.0 * T.a2) * th2) + (6.0 * T.a3) * th3) + (7.0 * T.a4) * th4;
        th = th - F / (th2 * dP);
    }
    double th2 = th * th, th4 = th2 * th2, th8 = th4 * th4;
    T.tc = (5.0 * T.M) / (eta * th8);
    T.th0 = th;
    T.M5 = 5.0 * T.M;
    T.M40 = 40.0 * T.M;
    T.r5M = 1.0 / T.M5;
    T.rc8 = 1.0 / T.c8;
    T.r40M = 1.0 / T.M40;
    T.reta = 1.0 / eta;
}

// Phase Phi (rad, phi_c = 0), GW frequency f and its derivative at time t < t_c, in the
// operation order of the formulas: q = eta (t_c - t) / (5M), theta = 1 / q^(1/8) (three correctly
// rounded square roots), f = (theta^3 / (8 pi M)) P_f, fdot = ((theta^2 / (8 pi M)) P_f') (eta theta^9 / (40M)),
// Phi = -(2 theta^-5 P_phi) / eta with theta^-5 = 1 / (theta^4 theta).  Divisions by the
// per-template constants 5M, 8 pi M, 40M and eta are formed by div_rn (the same correctly
// rounded quotients); 1/s and 1/(theta^4 theta) by rcp_rn and the roots by sqrt_pos (the same
// correctly rounded results: every caller has t_c - t > 0 with q, s and theta far inside the normal range).
// s_out, if given, receives s = 1/theta (the VJP's tangents reuse it).
__device__ inline void track_at(const Track &T, double t, double &Phi, double &f, double &fdot,
                                double *s_out = nullptr) {
    double tau = T.tc - t;
    double q = div_rn(T.eta * tau, T.M5, T.r5M);
    double s = sqrt_pos(sqrt_pos(sqrt_pos(q)));
    if (s_out) *s_out = s;
    double th = rcp_rn(s);
    double th2 = th * th, th3 = th2 * th, th4 = th2 * th2;
    double Pf = ((1.0 + T.a2 * th2) + T.a3 * th3) + T.a4 * th4;
    f = div_rn(th3, T.c8, T.rc8) * Pf;
    double dPf = ((3.0 + (5.0 * T.a2) * th2) + (6.0 * T.a3) * th3) + (7.0 * T.a4) * th4;
    double dfdth = div_rn(th2, T.c8, T.rc8) * dPf;
    double th8 = th4 * th4, th9 = th8 * th;
    double dthdt = div_rn(T.eta * th9, T.M40, T.r40M);
    fdot = dfdth * dthdt;
    double Pp = ((1.0 + T.b2 * th2) + T.b3 * th3) + T.b4 * th4;
    double thm5 = rcp_rn(th4 * th);
    Phi = -div_rn((2.0 * thm5) * Pp, T.eta, T.reta);
}

// Track end (paper Appendix A compactness + band edge + merger): returns 0 if
// tranche starting at tm is active, else the flag naming the condition.
__device__ __forceinline__ int track_step(const Track &T, double tm, double dT, double df, double fnyq,
                                          double &Phi, double &f, double &fdot) {
    if (tm + dT >= T.tc) return kFlagMergeEnd;
    track_at(T, tm, Phi, f, fdot);
    if ((f + fdot * dT >= fnyq - 11.0 * df) || (fdot * dT > 10.0 * df)) return kFlagBandEnd;
    return 0;
}

// track_step for the lanes of a wave: the track is evaluated unconditionally (past the merger it is NaN and
// the flag says so; the caller uses the values only where the flag is 0), which spares the wave the masked
// branch and the zeroed outputs.  Same flag and, where it is 0, the same values as track_step.
__device__ __forceinline__ int track_step_lanes(const Track &T, double tm, double dT, double df, double fnyq,
                                                double &Phi, double &f, double &fdot, double *s_out = nullptr) {
    track_at(T, tm, Phi, f, fdot, s_out);
    if (tm + dT >= T.tc) return kFlagMergeEnd;
    if ((f + fdot * dT >= fnyq - 11.0 * df) || (fdot * dT > 10.0 * df)) return kFlagBandEnd;
    return 0;
}

// N_seg rule: 16 * 2^n, n = number of thresholds 1.34e-12 * 2^(3i-2) * sqrt 2 that fdot0 reaches.
__device__ __forceinline__ int nseg_rule(double fdot0) {
    int n = 0;
    double r2 = sqrt(2.0);
    for (int i = 1; i <= 4; ++i)
        if (fdot0 >= kFdotRef * ldexp(r2, 3 * i - 2)) ++n;
    return 16 << n;
}

// x / (2 pi) reduced to [-1/2, 1/2] revolutions (FMA-based two-constant reduction).
__device__ __forceinline__ double phase_to_rev(double x) {
    const double hi = 6.283185307179586232;      // 2 pi rounded to double
    const double lo = 2.4492935982947064e-16;    // 2 pi - hi
    double n = rint(x * (1.0 / kTwoPi));
    double r = fma(-n, hi, x);
    r = fma(-n, lo, r);
    return r * (1.0 / kTwoPi);
}

__device__ __forceinline__ double frac_rev(double r) { return r - rint(r); }

// ------------------------------------------------------------------ complex helpers
template <class R>
struct cx {
    R re, im;
};
template <class R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
#pragma clang fp contract(fast)
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.re * s, a.im * s}; }

// e^{2 pi i r} for r in revolutions (|r| <= 1/2 after reduction).
__device__ __forceinline__ cx<double> expi_rev(double r) {
    double s, c;
    sincospi(2.0 * r, &s, &c);
    return {c, s};
}
__device__ __forceinline__ cx<float> expi_rev(float r) {
    // hardware sine/cosine take their argument in revolutions
    return {__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r)};
}
__device__ __forceinline__ double sin_rev(double r) { return sinpi(2.0 * r); }
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
// sin(2 pi r) for |r| <= 1/4 with relative (not only absolute) accuracy for small r.  FP32: the
// odd Taylor series of sin x through x^13 at x = 2 pi r (|x| <= pi/2, where the first omitted
// term is below 7e-10 and every partial sum keeps the sign of x); Horner form in x^2.
__device__ __forceinline__ double sin_rev_accurate(double r) { return sinpi(2.0 * r); }
__device__ __forceinline__ float sin_rev_accurate(float r) {
#pragma clang fp contract(fast)
    const float x = r * (float)kTwoPi;
    const float x2 = x * x;
    float p = 1.0f / 6227020800.0f;  // 1/13!
    p = p * x2 - 1.0f / 39916800.0f;  // 1/11!
    p = p * x2 + 1.0f / 362880.0f;    // 1/9!
    p = p * x2 - 1.0f / 5040.0f;      // 1/7!
    p = p * x2 + 1.0f / 120.0f;       // 1/5!
    p = p * x2 - 1.0f / 6.0f;         // 1/3!
    return x + (x * x2) * p;
}
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ------------------------------------------------------------------ response
// Per-tranche geometry table (FP64, structure of arrays, row stride Nt, so the 64
// lanes of a wave on consecutive tranches read 512 contiguous bytes per row): rows
// 0..8 spacecraft positions p_i (light-seconds), rows 9..17 unit arm vectors
// n_01, n_12, n_20 (from the first spacecraft to the second).
constexpr int kGeoRows = 18;

// Sky constants of one template.  With the sky basis u = (cos th cos phi, cos th sin phi,
// -sin th), v = (sin phi, -cos phi, 0) and an arm direction n, the arm's polarisation factor is
//   a_+ [cos 2psi (n.u^2 - n.v^2) + sin 2psi 2 n.u n.v] - i cos(iota) [-sin 2psi (...) + cos 2psi (...)],
// a_+ = (1 + cos^2 iota) / 2.  Rotating the basis by psi (u' = cos psi u + sin psi v,
// v' = -sin psi u + cos psi v) turns the two brackets into n.u'^2 - n.v'^2 and 2 n.u' n.v', and
// scaling u', v' by sqrt(a_+) leaves  (n.u''^2 - n.v''^2) + i q n.u'' n.v''  with
// q = -2 cos(iota) / a_+ : the same value with four fewer operations per arm and tranche.
template <class R>
struct Sky {
    R k[3], u[3], v[3];  // propagation direction; u'', v'' as above
    R q;
    double kd[3];
};

template <class R>
__device__ inline void sky_init(Sky<R> &S, double ct, double phi, double psi, double ci) {
    double st = sqrt(1.0 - ct * ct);
    double sp, cp, ss, cs;
    sincos(phi, &sp, &cp);
    sincos(psi, &ss, &cs);
    S.kd[0] = -st * cp;
    S.kd[1] = -st * sp;
    S.kd[2] = -ct;
    for (int i = 0; i < 3; ++i) S.k[i] = (R)S.kd[i];
    const double ap = (1.0 + ci * ci) / 2.0;
    const double ra = sqrt(ap);
    const double u[3] = {ct * cp, ct * sp, -st};
    const double v[3] = {sp, -cp, 0.0};
    for (int i = 0; i < 3; ++i) {
        S.u[i] = (R)(ra * (cs * u[i] + ss * v[i]));
        S.v[i] = (R)(ra * (cs * v[i] - ss * u[i]));
    }
    S.q = (R)(-2.0 * ci / ap);
}

// sin(2 pi y) / y = 2 pi sinc(2 pi y) for an argument y in revolutions (the hardware sine takes revolutions, so
// no scaling of the argument is spent; the constant 2 pi is folded into the caller's prefactor); series near 0,
// selected rather than branched on (the unselected quotient may be inf or nan at y = 0).
template <class R>
__device__ __forceinline__ R sinc_rev2pi(R y) {
#pragma clang fp contract(fast)
    const R q = sin_rev(y) * rcp(y);
    const R ser = (R)kTwoPi - y * y * (R)(kTwoPi * kTwoPi * kTwoPi / 6.0);
    return y < (R)1.6e-5 ? ser : q;
}

// Buffer views of the geometry tables: the FP64 table (rows of Nt doubles) and, for the FP32
// arithmetic, the FP32 copy of the arm-vector rows 9..17 (rows of Nt floats).  A value is
// read with the lane's tranche as vector offset and the row as scalar offset, so no vector
// address arithmetic is spent on it.
struct GeoView {
    __amdgpu_buffer_rsrc_t g64, g32;
    uint32_t row64, row32;  // bytes per row
    __amdgpu_buffer_rsrc_t lk;  // a caller's link light times [6][Nt] (FP64, rows of row64 bytes), if any
    int tdi2;                   // with the link table: second-generation TDI combinations
};

__device__ __forceinline__ GeoView geo_view(const double *geo, const float *geo32, int Nt,
                                            const double *links = nullptr, int tdi2 = 0) {
    GeoView v;
    v.row64 = (uint32_t)Nt * 8u;
    v.row32 = (uint32_t)Nt * 4u;
    v.g64 = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(geo), (short)0, (int)(v.row64 * kGeoRows), 0x00020000);
    v.g32 = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(geo32), (short)0, (int)(v.row32 * 9u), 0x00020000);
    v.lk = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(links), (short)0, links ? (int)(v.row64 * 6u) : 0,
                                             0x00020000);
    v.tdi2 = tdi2;
    return v;
}

__device__ __forceinline__ double geo_link(const GeoView &v, int m, int l) {  // light time of link row l
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v.lk, (uint32_t)m * 8u, (uint32_t)l * v.row64, 0));
}

__device__ __forceinline__ double geo_d(const GeoView &v, int m, int r) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v.g64, (uint32_t)m * 8u, (uint32_t)r * v.row64, 0));
}

template <class R>
__device__ __forceinline__ R geo_arm(const GeoView &v, int m, int q) {  // arm-vector value q = 0..8
    if constexpr (sizeof(R) == 4)
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(v.g32, (uint32_t)m * 4u, (uint32_t)q * v.row32, 0));
    else
        return geo_d(v, m, 9 + q);
}

__device__ __forceinline__ void load_geo(const double *__restrict__ geo, int m, int Nt, double g[kGeoRows]) {
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) g[r] = geo[(size_t)r * Nt + m];
}

// T_A, T_E at tranche m (time t_m) and frequency f from the geometry tables; each value
// is read where it is used, which keeps register pressure down.
template <class R, bool WITH_T = false>
__device__ inline void transfer_ae(const Sky<R> &S, const GeoView &gv, int m, double f, cx<R> &TA, cx<R> &TE,
                                   cx<R> *TT = nullptr) {
#pragma clang fp contract(fast)
    const double L = kArmM / kClight;
    double kp[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        kp[i] = S.kd[0] * geo_d(gv, m, 3 * i) + S.kd[1] * geo_d(gv, m, 3 * i + 1) + S.kd[2] * geo_d(gv, m, 3 * i + 2);
    const R hfL = (R)(0.5 * f * L);  // pi f L in revolutions
    // Arm a, direction (s -> r) and reverse: G = -i pi f L e^{i ph} amp sinc(pi f L (1 -+ k.n)); the sinc is
    // taken as 2 pi sinc (sinc_rev2pi), and the common factor -i pi f L / (2 pi) is applied once, to T_A and T_E.
    cx<R> Gd[3], Gr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int s = a, r = (a + 1) % 3;
        R n0 = geo_arm<R>(gv, m, 3 * a + 0);
        R n1 = geo_arm<R>(gv, m, 3 * a + 1);
        R n2 = geo_arm<R>(gv, m, 3 * a + 2);
        R kn = S.k[0] * n0 + S.k[1] * n1 + S.k[2] * n2;
        R nu = S.u[0] * n0 + S.u[1] * n1 + S.u[2] * n2;
        R nv = S.v[0] * n0 + S.v[1] * n1 + S.v[2] * n2;
        cx<R> amp = {nu * nu - nv * nv, S.q * (nu * nv)};
        double rev = frac_rev(-0.5 * f * (L + (kp[s] + kp[r])));  // -pi f (L + k.(p_s + p_r)) / 2 pi
        cx<R> E = expi_rev((R)rev);
        cx<R> Ea = cmul(E, amp);
        Gd[a] = cscale(Ea, sinc_rev2pi(hfL * ((R)1 - kn)));
        Gr[a] = cscale(Ea, sinc_rev2pi(hfL * ((R)1 + kn)));
    }
    // 0-based spacecraft: arm 0 = (0,1), arm 1 = (1,2), arm 2 = (2,0)
    const cx<R> G01 = Gd[0], G10 = Gr[0], G12 = Gd[1], G21 = Gr[1], G20 = Gd[2], G02 = Gr[2];
    // D = e^{-2 pi i f L};  1 - D^2 = 2 i sin(2 pi f L) D exactly.  The sine is taken of an
    // argument folded into [-1/4, 1/4] revolutions, so it keeps full relative precision at
    // the transfer nulls f = n / (2L) where 1 - D^2 computed directly would cancel.
    const double rl = frac_rev(f * L);
    cx<R> D = expi_rev((R)(-rl));
    const double rf = rl > 0.25 ? 0.5 - rl : (rl < -0.25 ? -0.5 - rl : rl);
    const R s2 = sin_rev_accurate((R)rf);
    // X = (1 - D^2)[(G20 - G10) + D (G02 - G01)] and cyclic; the common factor 1 - D^2 and the
    // 1/sqrt2, 1/sqrt6 of A and E are applied once to the combinations.
    const cx<R> Xp = cadd(csub(G20, G10), cmul(D, csub(G02, G01)));
    const cx<R> Yp = cadd(csub(G01, G21), cmul(D, csub(G10, G12)));
    const cx<R> Zp = cadd(csub(G12, G02), cmul(D, csub(G21, G20)));
    // (1 - D^2)(-i pi f L) / (2 pi) = sin(2 pi f L) f L D, times 1/sqrt2 (A) or 1/sqrt6 (E)
    const R is2 = (R)0.70710678118654752440, is6 = (R)0.40824829046386301637;
    const R sp = s2 * (hfL + hfL);
    const cx<R> oma = cscale(D, sp * is2);
    const cx<R> ome = cscale(D, sp * is6);
    TA = cmul(oma, csub(Zp, Xp));
    TE = cmul(ome, cadd(csub(Xp, cscale(Yp, (R)2)), Zp));
    if constexpr (WITH_T) {
        // the third channel T = (X + Y + Z) / sqrt3, the null channel of the equal-arm constellation
        const R is3 = (R)0.57735026918962576451;
        *TT = cmul(cscale(D, sp * is3), cadd(cadd(Xp, Yp), Zp));
    }
}

// T_A, T_E (and T) with the six link light times of the tranche from the caller's table (unequal arms; the
// two directions of an arm may differ, as with point-ahead), the geometry frozen over the tranche.  Table rows
// 0..2 are the links s = a -> r = a + 1 of arms a = 0..2, rows 3..5 their reverse links.  Link s -> r is
// received at p_r after travelling L_sr along the arm direction n_sr, so it left from p_r - L_sr n_sr:
//   G_sr = -i pi f L_sr sinc(pi f L_sr (1 - k.n_sr)) e^{-i pi f (L_sr (1 - k.n_sr) + 2 k.p_r)} amp_a,
// and first-generation TDI with each path's delay D_sr = e^{-2 pi i f L_sr}:
//   X = (1 - D01 D10)(G20 + D20 G02) - (1 - D02 D20)(G10 + D10 G01), Y and Z cyclic.
// The round trip of arm a, l_a = L_sr + L_rs, enters as 1 - D_sr D_rs = 2 i sin(pi f l_a) e^{-i pi f l_a}
// (the sine of an argument folded into [-1/4, 1/4] revolutions, as for equal arms); with the common factor
// -i pi f it is the real 2 pi f sin(pi f l_a) times e^{-i pi f l_a}, of which 2 pi goes into the sincs
// (sinc_rev2pi) and f sin(pi f l_a) e^{-i pi f l_a} stays in F.  f k.p_r reaches tens of revolutions and
// is reduced in FP64; the link terms below a revolution are formed in R.
// Second generation (gv.tdi2, the arms static over the tranche): each combination minus itself delayed by the
// round trips of its two arms, X2 = (1 - R_0 R_2) X, Y2 = (1 - R_0 R_1) Y, Z2 = (1 - R_1 R_2) Z with
// R_a = e^{-2 pi i f l_a}, each factor formed as 2 i sin(pi f (l_a + l_b)) e^{-i pi f (l_a + l_b)}.
template <class R>
__device__ __forceinline__ cx<R> one_minus_round_trips(double f, double lab) {
    const double rr = frac_rev(0.5 * f * lab);
    const double rfold = rr > 0.25 ? 0.5 - rr : (rr < -0.25 ? -0.5 - rr : rr);
    const R s2 = (R)2 * sin_rev_accurate((R)rfold);
    const cx<R> e = expi_rev((R)(-rr));
    return {-s2 * e.im, s2 * e.re};
}

template <class R, bool WITH_T = false>
__device__ inline void transfer_links(const Sky<R> &S, const GeoView &gv, int m, double f, cx<R> &TA, cx<R> &TE,
                                      cx<R> *TT = nullptr) {
#pragma clang fp contract(fast)
    R rp[3];  // -f k.p_i in revolutions, reduced
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double kp =
            S.kd[0] * geo_d(gv, m, 3 * i) + S.kd[1] * geo_d(gv, m, 3 * i + 1) + S.kd[2] * geo_d(gv, m, 3 * i + 2);
        rp[i] = (R)frac_rev(-f * kp);
    }
    const R hp = (R)(0.5 * f), hf = -hp, rf = (R)f;
    cx<R> Gd[3], Gr[3], F[3], Dd[3], Dr[3];
    double la[3];  // round trips of the arms
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int s = a, r = (a + 1) % 3;
        const double Lfd = geo_link(gv, m, a), Lbd = geo_link(gv, m, 3 + a);
        la[a] = Lfd + Lbd;
        const R Lf = (R)Lfd, Lb = (R)Lbd;
        R n0 = geo_arm<R>(gv, m, 3 * a + 0);
        R n1 = geo_arm<R>(gv, m, 3 * a + 1);
        R n2 = geo_arm<R>(gv, m, 3 * a + 2);
        R kn = S.k[0] * n0 + S.k[1] * n1 + S.k[2] * n2;
        R nu = S.u[0] * n0 + S.u[1] * n1 + S.u[2] * n2;
        R nv = S.v[0] * n0 + S.v[1] * n1 + S.v[2] * n2;
        cx<R> amp = {nu * nu - nv * nv, S.q * (nu * nv)};
        const R om = (R)1 - kn, op = (R)1 + kn;  // 1 - k.n of the forward and of the reverse link
        const cx<R> Ef = expi_rev(rp[r] + hf * Lf * om);
        const cx<R> Eb = expi_rev(rp[s] + hf * Lb * op);
        // the sincs as 2 pi sinc of arguments in revolutions; the 1 / (2 pi) goes into F below
        Gd[a] = cscale(cmul(Ef, amp), Lf * sinc_rev2pi(hp * Lf * om));
        Gr[a] = cscale(cmul(Eb, amp), Lb * sinc_rev2pi(hp * Lb * op));
        Dd[a] = expi_rev(-(rf * Lf));
        Dr[a] = expi_rev(-(rf * Lb));
        const double rr = frac_rev(0.5 * f * la[a]);
        const double rfold = rr > 0.25 ? 0.5 - rr : (rr < -0.25 ? -0.5 - rr : rr);
        F[a] = cscale(expi_rev((R)(-rr)), rf * sin_rev_accurate((R)rfold));
    }
    // 0-based spacecraft: arm 0 = (0,1), arm 1 = (1,2), arm 2 = (2,0)
    const cx<R> G01 = Gd[0], G10 = Gr[0], G12 = Gd[1], G21 = Gr[1], G20 = Gd[2], G02 = Gr[2];
    const cx<R> D01 = Dd[0], D10 = Dr[0], D12 = Dd[1], D21 = Dr[1], D20 = Dd[2], D02 = Dr[2];
    cx<R> X = csub(cmul(F[0], cadd(G20, cmul(D20, G02))), cmul(F[2], cadd(G10, cmul(D10, G01))));
    cx<R> Y = csub(cmul(F[1], cadd(G01, cmul(D01, G10))), cmul(F[0], cadd(G21, cmul(D21, G12))));
    cx<R> Z = csub(cmul(F[2], cadd(G12, cmul(D12, G21))), cmul(F[1], cadd(G02, cmul(D02, G20))));
    if (gv.tdi2) {
        X = cmul(one_minus_round_trips<R>(f, la[0] + la[2]), X);
        Y = cmul(one_minus_round_trips<R>(f, la[0] + la[1]), Y);
        Z = cmul(one_minus_round_trips<R>(f, la[1] + la[2]), Z);
    }
    const R is2 = (R)0.70710678118654752440, is6 = (R)0.40824829046386301637;
    TA = cscale(csub(Z, X), is2);
    TE = cscale(cadd(csub(X, cscale(Y, (R)2)), Z), is6);
    if constexpr (WITH_T) {
        const R is3 = (R)0.57735026918962576451;
        *TT = cscale(cadd(cadd(X, Y), Z), is3);
    }
}

// ------------------------------------------------------------------ tranche spectrum
// Per-tranche constants of the Fresnel-kernel spectrum in bin units.  With
// x = f_m dT - k_c in (-1, 0], beta = fdot dT^2 and s = sqrt(2 / beta), the
// Fresnel arguments of bin k = k_c + j are v0 = s (x - j), v1 = s (x - j + beta),
// and since f_k dT is an integer, Eq. (fresnel-ft) becomes
//   h_j = P { (sgn v1 - sgn v0) (1+i)/2 e^{i(phi_m - pi (x-j)^2 / beta)}
//             - sgn v1 (g1 + i f1) e^{i phi_end} + sgn v0 (g0 + i f0) e^{i phi_m} },
// P = A / sqrt(2 fdot), phi_end = phi_m + 2 pi x + pi beta, using
// C(z) + i S(z) = sgn z [(1+i)/2 - (g(|z|) + i f(|z|)) e^{i pi z^2 / 2}] with
// the paper's f, g (rational for |z| <= 6, f = 1/(pi |z|), g = 0 above).  When
// both |v| > 6 and no bin frequency is crossed this is
//   h_j = i Q (e^{i phi_m} / (x - j) - e^{i phi_end} / (x - j + beta)),  Q = A dT / (2 pi).
//
// The paper's Fresnel forms jump at |z| = 6 (by up to ~5e-4), so which branch a bin edge
// takes is an integer decision and is made in FP64 for every precision: |v0| <= 6 exactly
// for j in [j0lo, j0hi] and |v1| <= 6 for j in [j1lo, j1hi] (computed from FP64 x, beta
// and r6 = 6 / s).  A bin is in the asymptotic-only region exactly when j < j0lo or
// j > j1hi.
template <class R>
struct TrancheSpec {
    R x, beta, s, P, Q, half_inv_beta;
    cx<R> E0, E1;
    double rev0;  // phi_m in revolutions, reduced
    int j0lo, j0hi, j1lo, j1hi;
};

template <class R>
__device__ __forceinline__ bool bin_is_fast(const TrancheSpec<R> &ts, int j) {
    return j < ts.j0lo || j > ts.j1hi;
}

template <class R>
__device__ __forceinline__ void fresnel_fg(R av, bool rational, R &f, R &g) {
#pragma clang fp contract(fast)
    if (!rational) {
        f = rcp((R)kPi * av);
        g = (R)0;
    } else {
        R a2 = av * av;
        f = ((R)1 + (R)0.926 * av) * rcp((R)2 + (R)1.792 * av + (R)3.104 * a2);
        g = rcp((R)2 + (R)4.142 * av + (R)3.492 * a2 + (R)6.670 * a2 * av);
    }
}

// Fresnel modes of the tranche spectrum: the paper's two-branch forms, or the Fresnel integrals themselves.
enum : int { kFresnelPaper = 0, kFresnelAccurate = 1 };

// The auxiliary functions f(z), g(z) of the Fresnel integrals, C(z) + i S(z) = (1+i)/2 - (g + i f) e^{i pi z^2/2}
// for z >= 0, to FP64 rounding (for the accurate Fresnel mode):
// * z <= 1.8: the power series of C and S (terms z x^k / k!, x = pi z^2 / 2, 40 terms), then
//   f = (1/2 - S) cos x - (1/2 - C) sin x and g = (1/2 - C) cos x + (1/2 - S) sin x;
// * 1.8 < z < 6: g + i f = (1+i)/2 e^{w^2} erfc(w) at w = (sqrt(pi)/2)(1 - i) z, with e^{w^2} erfc(w) from its
//   continued fraction 1 / (sqrt(pi) (w + (1/2) / (w + 1 / (w + (3/2) / (w + ...))))), 64 levels;
// * z >= 6: the asymptotic series f ~ (1/(pi z)) sum (-1)^m (4m-1)!! / (pi z^2)^(2m),
//   g ~ (1/(pi^2 z^3)) sum (-1)^m (4m+1)!! / (pi z^2)^(2m), nine terms.
__device__ inline void fresnel_fg_accurate(double z, double &f, double &g) {
    if (z <= 1.8) {
        const double x = 0.5 * kPi * z * z;
        double t = z, C = 0.0, S = 0.0;
#pragma unroll 4
        for (int k = 0; k < 40; ++k) {
            const double term = t / (double)(2 * k + 1);
            const double sg = ((k >> 1) & 1) ? -1.0 : 1.0;
            if (k & 1)
                S += sg * term;
            else
                C += sg * term;
            t *= x / (double)(k + 1);
        }
        double sx, cx_;
        sincos(x, &sx, &cx_);
        f = (0.5 - S) * cx_ - (0.5 - C) * sx;
        g = (0.5 - C) * cx_ + (0.5 - S) * sx;
    } else if (z < 6.0) {
        const double a = 0.8862269254527580 * z;  // sqrt(pi)/2 z: w = a - i a
        double dr = a, di = -a;
        for (int n = 64; n >= 1; --n) {
            const double q = (0.5 * n) / (dr * dr + di * di);
            const double nr = a + q * dr, ni = -a - q * di;  // w + (n/2) / d
            dr = nr;
            di = ni;
        }
        // e = 1 / (sqrt(pi) d); (g + i f) = (1 + i)/2 e
        const double den = 1.7724538509055160 * (dr * dr + di * di);
        const double er = dr / den, ei = -di / den;
        g = 0.5 * (er - ei);
        f = 0.5 * (er + ei);
    } else {
        const double pz2 = kPi * z * z;
        const double y = 1.0 / (pz2 * pz2);
        double cf = 1.0, cg = 1.0, sf = 1.0, sg = 1.0, ym = 1.0;
        for (int m = 1; m <= 8; ++m) {
            cf *= (double)((4 * m - 3) * (4 * m - 1));
            cg *= (double)((4 * m - 1) * (4 * m + 1));
            ym *= -y;
            sf += cf * ym;
            sg += cg * ym;
        }
        f = sf / (kPi * z);
        g = sg / (kPi * pz2 * z);
    }
}

// Asymptotic Fresnel on both tranche edges and no bin frequency crossed (bin_is_fast):
// h_j = i Q (e^{i phi_m}/(x - j) - e^{i phi_end}/(x - j + beta)).
template <class R>
__device__ __forceinline__ cx<R> bin_fast(const TrancheSpec<R> &ts, R xj) {
#pragma clang fp contract(fast)
    const R xj1 = xj + ts.beta;
    R a, b;
    if constexpr (sizeof(R) == 4) {
        // one hardware reciprocal for both: 1/xj = xj1 r, 1/xj1 = xj r with r = 1/(xj xj1)
        const R r = rcp(xj * xj1);
        a = xj1 * r;
        b = xj * r;
    } else {
        a = rcp(xj);
        b = rcp(xj1);
    }
    R re = ts.E0.re * a - ts.E1.re * b;
    R im = ts.E0.im * a - ts.E1.im * b;
    return {-ts.Q * im, ts.Q * re};
}

// General form, valid for every bin j (both Fresnel branches, stationary-phase term).  FR = kFresnelAccurate
// takes the Fresnel integrals' own f, g (FP64) in place of the paper's forms.
template <class R, int FR = kFresnelPaper>
__device__ __forceinline__ cx<R> bin_full(const TrancheSpec<R> &ts, R xj, int j) {
#pragma clang fp contract(fast)
    R xj1 = xj + ts.beta;
    R v0 = ts.s * xj, v1 = ts.s * xj1;
    R f0, g0, f1, g1;
    if constexpr (FR == kFresnelAccurate) {
        double a, b;
        fresnel_fg_accurate((double)fabs(v0), a, b);
        f0 = (R)a;
        g0 = (R)b;
        fresnel_fg_accurate((double)fabs(v1), a, b);
        f1 = (R)a;
        g1 = (R)b;
    } else {
        fresnel_fg(fabs(v0), j >= ts.j0lo && j <= ts.j0hi, f0, g0);
        fresnel_fg(fabs(v1), j >= ts.j1lo && j <= ts.j1hi, f1, g1);
    }
    // The sign of each Fresnel argument is its sign bit (an argument of exactly 0 counts as positive: since
    // f(0) = g(0) = 1/2, the edge term (1+i)/2 e^{i phi} it then adds is the stationary-phase term it removes,
    // so the value is the same as with sgn 0 there).
    cx<R> t0 = cmul(cx<R>{copysign(g0, v0), copysign(f0, v0)}, ts.E0);
    cx<R> t1 = cmul(cx<R>{copysign(g1, v1), copysign(f1, v1)}, ts.E1);
    cx<R> h = csub(t0, t1);
    if (std::signbit(v0) != std::signbit(v1)) {
        // bin frequency crossed inside the tranche: stationary-phase term, (sgn v1 - sgn v0) / 2 = +-1
        double rv = frac_rev(ts.rev0 - (double)(xj * xj * ts.half_inv_beta));
        cx<R> e = expi_rev((R)rv);
        const R hh = std::signbit(v0) ? (R)1 : (R)-1;
        h.re += hh * (e.re - e.im);
        h.im += hh * (e.re + e.im);
    }
    return cscale(h, ts.P);
}

// h_j w for a bin in the asymptotic region, with the weight w folded into the reciprocals.
template <class R>
__device__ __forceinline__ cx<R> bin_fast_weighted(const TrancheSpec<R> &ts, R xj, R w) {
#pragma clang fp contract(fast)
    const R xj1 = xj + ts.beta;
    const R qw = ts.Q * w;
    R a, b;
    if constexpr (sizeof(R) == 4) {
        const R r = rcp(xj * xj1) * qw;
        a = xj1 * r;
        b = xj * r;
    } else {
        a = qw / xj;
        b = qw / xj1;
    }
    const R re = ts.E0.re * a - ts.E1.re * b;
    const R im = ts.E0.im * a - ts.E1.im * b;
    return {-im, re};
}

// h_j w for bin k_c + j: asymptotic form where both Fresnel arguments exceed 6 and no bin
// frequency is crossed, the general form otherwise (always, in the accurate Fresnel mode).
template <class R, int FR = kFresnelPaper>
__device__ __forceinline__ cx<R> tranche_bin_weighted(const TrancheSpec<R> &ts, int j, R w) {
    R xj = ts.x - (R)j;
    if (FR == kFresnelPaper && bin_is_fast(ts, j)) return bin_fast_weighted(ts, xj, w);
    const cx<R> h = bin_full<R, FR>(ts, xj, j);
    return {h.re * w, h.im * w};
}

template <class R>
__device__ __forceinline__ cx<R> tranche_spectrum_bin(const TrancheSpec<R> &ts, int j) {
    R xj = ts.x - (R)j;
    if (bin_is_fast(ts, j)) return bin_fast(ts, xj);
    return bin_full(ts, xj, j);
}

// Tranche constants from the FP64 track.  Returns k_c.  Bin index, offset and
// phases come from FP64; the rest is formed in R.  The amplitude is A = f_amp^(2/3); f_amp < 0 takes
// f itself (a harmonic of a multi-harmonic template passes the dominant harmonic's frequency).
template <class R>
__device__ __forceinline__ int tranche_setup(TrancheSpec<R> &ts, double Phi, double f, double fdot, double dT,
                                             double f_amp = -1.0) {
    const double fa = f_amp < 0.0 ? f : f_amp;
    double fT = f * dT;
    double kc = ceil(fT);
    double x = fT - kc;
    double beta = (fdot * dT) * dT;
    double rev0 = phase_to_rev(Phi);
    double rev1 = frac_rev(rev0 + x + 0.5 * beta);
    ts.x = (R)x;
    ts.beta = (R)beta;
    {
        // rational-branch bin ranges of the two edges, decided in FP64 (|v| <= 6 is rational)
        const double r6 = sqrt(18.0 * beta);  // 6 / s with s = sqrt(2 / beta)
        ts.j0lo = (int)ceil(x - r6);
        ts.j0hi = (int)floor(x + r6);
        ts.j1lo = (int)ceil((x + beta) - r6);
        ts.j1hi = (int)floor((x + beta) + r6);
    }
    if constexpr (sizeof(R) == 8) {
        ts.s = sqrt(2.0 / beta);
        double A = pow(fa, 2.0 / 3.0);
        ts.P = A / sqrt(2.0 * fdot);
        ts.Q = A * dT / kTwoPi;
        ts.half_inv_beta = 0.5 / beta;
    } else {
        float b = (float)beta;
        float ib = rcp(b);
        ts.s = sqrtf(2.0f * ib);
        float A = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)fa) * (2.0f / 3.0f));
        ts.P = A * __builtin_amdgcn_rsqf((float)(2.0 * fdot));
        ts.Q = A * (float)(dT / kTwoPi);
        ts.half_inv_beta = 0.5f * ib;
    }
    ts.E0 = expi_rev((R)rev0);
    ts.E1 = expi_rev((R)rev1);
    ts.rev0 = rev0;
    return (int)kc;
}

// ------------------------------------------------------------------ pixel loads
template <class PixT>
struct PixTraits;
template <>
struct PixTraits<double> {
    using R = double;
    static constexpr bool scaled = false;
    __device__ static __forceinline__ cx<double> load(const void *p, size_t idx) {
        double2 v = reinterpret_cast<const double2 *>(p)[idx];
        return {v.x, v.y};
    }
};
template <>
struct PixTraits<float> {
    using R = float;
    static constexpr bool scaled = false;
    __device__ static __forceinline__ cx<float> load(const void *p, size_t idx) {
        float2 v = reinterpret_cast<const float2 *>(p)[idx];
        return {v.x, v.y};
    }
};
template <>
struct PixTraits<__half> {
    using R = float;
    static constexpr bool scaled = true;
    __device__ static __forceinline__ cx<float> load(const void *p, size_t idx) {
        __half2 v = reinterpret_cast<const __half2 *>(p)[idx];
        float2 f = __half22float2(v);
        return {f.x, f.y};
    }
};
// complex int16 fixed point: the low half of the 32-bit word is the real part
__device__ __forceinline__ cx<float> i16x2_to_float(uint32_t w) {
    return {(float)(int)(int16_t)(w & 0xffffu), (float)((int)w >> 16)};
}
template <>
struct PixTraits<int16_t> {
    using R = float;
    static constexpr bool scaled = true;
    __device__ static __forceinline__ cx<float> load(const void *p, size_t idx) {
        return i16x2_to_float(reinterpret_cast<const uint32_t *>(p)[idx]);
    }
};
template <>
struct PixTraits<__hip_bfloat16> {
    using R = float;
    static constexpr bool scaled = true;
    __device__ static __forceinline__ cx<float> load(const void *p, size_t idx) {
        uint32_t w = reinterpret_cast<const uint32_t *>(p)[idx];
        return {__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
    }
};

}  // namespace tfsc
