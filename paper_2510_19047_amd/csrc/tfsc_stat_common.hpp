// Shared pieces of the statistic kernels: argument block, segment accumulation, tranche sums of the two
// schedules, wave-wide DPP reductions, and the kernel bodies, so that the kernel variants (the paper's
// Fresnel forms, the accurate Fresnel integrals, several harmonics) instantiate one implementation.
#pragma once

#include <limits.h>

#include "tfsc_device.hpp"
#include "tfsc_kernels.hpp"

namespace tfsc {

__global__ void k_zero_u32(uint32_t *p, int n);

// ------------------------------------------------------------------ common pieces
struct StatArgs {
    int M, K, Nt, C;
    double dt, dT, df, fnyq;
    const void *pix;
    uint32_t pix_bytes;  // size of the pixel store (WAVE schedule: < 4 GiB)
    const float *layer_scale;
    const double *inv_asd;
    const double *tranche_w;
    const double *geo;
    const float *geo32;
    const double *u_scale;  // [1], see k_weight_scale
    const float *rho;       // [K][Nt] per-pixel weight factor (general per-tranche PSD), else NULL
    uint32_t rho_bytes;
    const double *links;    // [6][Nt] link light times (unequal arms), else NULL
    int tdi2;               // with links: second-generation TDI combinations
    int64_t n;
    const double *mc, *eta, *f0, *ct, *phi, *psi, *ci;
    const int32_t *nseg;
    const int64_t *seg_offset;
    const int32_t *order;
    double *seg_terms, *stat, *seg_zn;
    int32_t *flags;
    int32_t *n_active;
    uint32_t *counter;
    // several noise realisations of the same grid (k_stat_wave_multi): realisation r's store
    // lies r * real_stride bytes after pix; its outputs at stat[r * n], seg_terms[r * seg_stride]
    uint32_t real_stride;
    int64_t seg_stride;
    int rho0;  // first realisation of this launch
};

// Chirp mass of template i: from the bank's mc, or exp(ln Mc) when the bank is given in ln Mc (the
// small per-template kernels; the statistic and VJP kernels read a table the entry point fills).
__device__ __forceinline__ double bank_mc(const double *mc, const double *ln_mc, int64_t i) {
    return ln_mc ? exp(ln_mc[i]) : mc[i];
}

template <class R>
struct SegAcc {
    double zr, zi, N, total;
    int cur;
    bool any;
};

// close segments [acc.cur, upto) writing Upsilon_n and (z_n, N_n)
__device__ __forceinline__ void close_segments(SegAcc<double> &acc, int upto, int64_t off, double *seg_terms,
                                               double *seg_zn, bool writer) {
    while (acc.cur < upto) {
        double v = acc.N > 0.0 ? 2.0 * (acc.zr * acc.zr + acc.zi * acc.zi) / acc.N : 0.0;
        if (writer) {
            seg_terms[off + acc.cur] = v;
            if (seg_zn) {
                seg_zn[3 * (off + acc.cur) + 0] = acc.zr;
                seg_zn[3 * (off + acc.cur) + 1] = acc.zi;
                seg_zn[3 * (off + acc.cur) + 2] = acc.N;
            }
        }
        if (acc.N > 0.0) acc.any = true;
        acc.total += v;
        acc.zr = acc.zi = acc.N = 0.0;
        ++acc.cur;
    }
}

// Segment boundaries b_s = ceil(s Nt / N_seg) stepped without division: tranche m lies in
// segment s = floor(m N_seg / Nt) exactly when b_s <= m < b_{s+1}.  The state (s Nt =
// qs N_seg + rs) advances by (q, r) = divmod(Nt, N_seg) per segment.
struct SegWalk {
    int s, lo, hi;      // current segment and its tranche range [lo, hi)
    int q, r, ns;       // divmod(Nt, N_seg), N_seg
    int qs, rs;         // (s + 1) Nt = qs N_seg + rs
    __device__ __forceinline__ void init(int Nt, int nseg) {
        ns = nseg;
        q = Nt / nseg;
        r = Nt - q * nseg;
        s = 0;
        lo = 0;
        qs = q;
        rs = r;
        hi = qs + (rs > 0 ? 1 : 0);
    }
    __device__ __forceinline__ void step() {
        ++s;
        lo = hi;
        qs += q;
        rs += r;
        if (rs >= ns) {
            qs += 1;
            rs -= ns;
        }
        hi = qs + (rs > 0 ? 1 : 0);
    }
};

// Sum over the 21 bins of tranche m: P_c = sum conj(D_ck) h_k u_k, Q = sum |h_k u_k|^2.
template <int C, class R, class PixT, int LAYOUT, class U, bool RHO, int FR = kFresnelPaper>
__device__ __forceinline__ void tranche_bins(const StatArgs &a, const TrancheSpec<R> &ts, int kc, int m,
                                             const U *__restrict__ u_tab, U u_mul, const float *__restrict__ sc_tab,
                                             cx<R> (&P)[C], R &Q) {
#pragma clang fp contract(fast)
    using PT = PixTraits<PixT>;
#pragma unroll
    for (int c = 0; c < C; ++c) P[c] = {(R)0, (R)0};
    Q = (R)0;
    const int kmax = a.M / 2 - 1;
#pragma unroll 3
    for (int j = -kHalfBins; j <= kHalfBins; ++j) {
        int k = kc + j;
        if (k < 1 || k > kmax) continue;
        R wk = (R)(u_tab[k] * u_mul);
        if constexpr (RHO) wk *= (R)a.rho[(size_t)k * a.Nt + m];
        const cx<R> g = tranche_bin_weighted<R, FR>(ts, j, wk);
        Q += g.re * g.re;
        Q += g.im * g.im;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            size_t idx = LAYOUT == 0   ? ((size_t)(c * a.K + k) * a.Nt + m)
                         : LAYOUT == 1 ? ((size_t)(c * a.Nt + m) * a.K + k)
                                       : ((size_t)k * a.Nt + m) * C + c;
            const auto Dl = PT::load(a.pix, idx);
            cx<R> D = {(R)Dl.re, (R)Dl.im};
            if constexpr (PT::scaled) {
                R s = (R)sc_tab[c * a.K + k];
                D.re *= s;
                D.im *= s;
            }
            P[c].re += D.re * g.re;
            P[c].re += D.im * g.im;
            P[c].im += D.re * g.im;
            P[c].im -= D.im * g.re;
        }
    }
}

// The response T_c(t_m, f_m) of the C channels.  LK: with the caller's link light times (unequal arms).
template <int C, class R, bool LK = false>
__device__ __forceinline__ void tranche_transfer(const Sky<R> &S, const GeoView &gv, int m, double f, cx<R> (&T)[C]) {
    cx<R> TA, TE, TT;
    if constexpr (LK)
        transfer_links<R, (C == 3)>(S, gv, m, f, TA, TE, &TT);
    else
        transfer_ae<R, (C == 3)>(S, gv, m, f, TA, TE, &TT);
    T[0] = TA;
    if constexpr (C >= 2) T[1] = TE;
    if constexpr (C == 3) T[2] = TT;
}

// Tranche contribution z_m = w_m sum_c T_c P_c, N_m = w_m^2 (sum_c |T_c|^2) Q.
template <int C, class R>
__device__ __forceinline__ void tranche_sums(const cx<R> (&T)[C], R wm, const cx<R> (&P)[C], R Q, R &zr, R &zi,
                                             R &nn) {
#pragma clang fp contract(fast)
    cx<R> z = cmul(T[0], P[0]);
    R tt = T[0].re * T[0].re + T[0].im * T[0].im;
    if constexpr (C >= 2) {
        z = cadd(z, cmul(T[1], P[1]));
        tt += T[1].re * T[1].re + T[1].im * T[1].im;
    }
    if constexpr (C == 3) {
        z = cadd(z, cmul(T[2], P[2]));
        tt += T[2].re * T[2].re + T[2].im * T[2].im;
    }
    zr = wm * z.re;
    zi = wm * z.im;
    nn = wm * wm * tt * Q;
}

template <int C, class R, bool LK = false>
__device__ __forceinline__ void tranche_combine(const Sky<R> &S, const GeoView &gv, int m, double f, R wm,
                                                const cx<R> (&P)[C], R Q, R &zr, R &zi, R &nn) {
    cx<R> T[C];
    tranche_transfer<C, R, LK>(S, gv, m, f, T);
    tranche_sums<C, R>(T, wm, P, Q, zr, zi, nn);
}

// ------------------------------------------------------------------ WAVE schedule
// Wave-wide sum of a float or double, result in every lane's scalar view (DPP row
// shifts within 16-lane rows, then row broadcasts 15 and 31; lane 63 ends with the
// total).  Called only in converged control flow.
__device__ __forceinline__ float dpp_sum_f32(float v) {
#pragma clang fp contract(fast)
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x112, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xf, 0xf, true));
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xf, 0xf, true));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

template <int CTRL, int RM, int BM>
__device__ __forceinline__ double dpp_add_step_f64(double v) {
    long long bits = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffffLL), CTRL, RM, BM, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, RM, BM, true);
    long long o = ((long long)(unsigned)lo) | ((long long)hi << 32);
    return v + __builtin_bit_cast(double, o);
}

__device__ __forceinline__ double dpp_sum_f64(double v) {
    // the two 32-bit halves move by DPP; the adds are FP64.  Full masks as in wave_sum3: only
    // lane 63's total is read, and a source outside the row reads +0.0.
    v = dpp_add_step_f64<0x111, 0xf, 0xf>(v);
    v = dpp_add_step_f64<0x112, 0xf, 0xf>(v);
    v = dpp_add_step_f64<0x114, 0xf, 0xf>(v);
    v = dpp_add_step_f64<0x118, 0xf, 0xf>(v);
    v = dpp_add_step_f64<0x142, 0xf, 0xf>(v);
    v = dpp_add_step_f64<0x143, 0xf, 0xf>(v);
    long long bits = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), 63);
    int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
    return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}

__device__ __forceinline__ float dpp_max_f32(float v) {
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, true)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x112, 0xf, 0xf, true)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xf, 0xe, true)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xf, 0xc, true)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xa, 0xf, true)));
    v = fmaxf(v, __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xc, 0xf, true)));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

template <int CTRL, int RM, int BM>
__device__ __forceinline__ void dpp_max_step2(int &a, int &b) {
    const int ta = __builtin_amdgcn_update_dpp(INT_MIN, a, CTRL, RM, BM, false);
    const int tb = __builtin_amdgcn_update_dpp(INT_MIN, b, CTRL, RM, BM, false);
    a = max(a, ta);
    b = max(b, tb);
}

// Wave-wide maxima of two ints (lane 63 holds both after the row shifts and broadcasts),
// interleaved so the two DPP moves of each step fill each other's hazard slots.
__device__ __forceinline__ void wave_max2_i32(int &a, int &b) {
    dpp_max_step2<0x111, 0xf, 0xf>(a, b);
    dpp_max_step2<0x112, 0xf, 0xf>(a, b);
    dpp_max_step2<0x114, 0xf, 0xe>(a, b);
    dpp_max_step2<0x118, 0xf, 0xc>(a, b);
    dpp_max_step2<0x142, 0xa, 0xf>(a, b);
    dpp_max_step2<0x143, 0xc, 0xf>(a, b);
    a = __builtin_amdgcn_readlane(a, 63);
    b = __builtin_amdgcn_readlane(b, 63);
}

template <class R>
__device__ __forceinline__ R wave_sum(R v) {
    if constexpr (sizeof(R) == 4) return dpp_sum_f32(v);
    else return dpp_sum_f64(v);
}

template <int CTRL, int RM, int BM>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, RM, BM, true));
}

template <int CTRL, int RM, int BM>
__device__ __forceinline__ void dpp_step3(float &a, float &b, float &c) {
    const float ta = dpp_f32<CTRL, RM, BM>(a), tb = dpp_f32<CTRL, RM, BM>(b), tc = dpp_f32<CTRL, RM, BM>(c);
    a += ta;
    b += tb;
    c += tc;
}

// Three wave sums at once: the three independent DPP moves of each step fill each other's
// data-hazard slots.  Only lane 63's total is read, so every step runs with full row and bank
// masks: a source outside the row reads 0 (bound_ctrl), lane 63 sees the same additions in the
// same order as with the masked inclusive scan, and each step folds into one DPP add.
template <class R>
__device__ __forceinline__ void wave_sum3(R &a, R &b, R &c) {
    if constexpr (sizeof(R) == 4) {
        dpp_step3<0x111, 0xf, 0xf>(a, b, c);
        dpp_step3<0x112, 0xf, 0xf>(a, b, c);
        dpp_step3<0x114, 0xf, 0xf>(a, b, c);
        dpp_step3<0x118, 0xf, 0xf>(a, b, c);
        dpp_step3<0x142, 0xf, 0xf>(a, b, c);
        dpp_step3<0x143, 0xf, 0xf>(a, b, c);
        a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, a), 63));
        b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, b), 63));
        c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, c), 63));
    } else {
        a = dpp_sum_f64(a);
        b = dpp_sum_f64(b);
        c = dpp_sum_f64(c);
    }
}

// Raw buffer view of the pixel store: hardware-checked, loads past the end return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pix_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <class PixT>
__device__ __forceinline__ cx<typename PixTraits<PixT>::R> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(PixT) == 8) {
        auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        double2 d = __builtin_bit_cast(double2, v);
        return {d.x, d.y};
    } else if constexpr (sizeof(PixT) == 4) {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        float2 f = __builtin_bit_cast(float2, v);
        return {f.x, f.y};
    } else {
        uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        if constexpr (sizeof(PixT) == 2 && PixTraits<PixT>::scaled && __is_same(PixT, __half)) {
            __half2 h = __builtin_bit_cast(__half2, w);
            float2 f = __half22float2(h);
            return {f.x, f.y};
        } else if constexpr (__is_same(PixT, int16_t)) {
            return i16x2_to_float(w);
        } else {
            return {__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u)};
        }
    }
}

// The C channel pixels of one bin: LAYER_MAJOR holds channel c at the scalar offset c * chan
// from channel 0, LAYER_MAJOR_CI holds the C pixels of a bin side by side, fetched with one
// wide load (two for FP64 pairs).
template <int C, class PixT, int LAYOUT>
__device__ __forceinline__ void bin_pixels(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t chan,
                                           cx<typename PixTraits<PixT>::R> (&D)[C]) {
    if constexpr (LAYOUT == 2 && C == 2) {
        if constexpr (sizeof(PixT) == 8) {
            const double2 d0 = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
            const double2 d1 = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + 16u, 0));
            D[0] = {d0.x, d0.y};
            D[1] = {d1.x, d1.y};
        } else if constexpr (sizeof(PixT) == 4) {
            const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
            D[0] = {q.x, q.y};
            D[1] = {q.z, q.w};
        } else {
            const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
            const uint32_t w0 = (uint32_t)w[0], w1 = (uint32_t)w[1];
            if constexpr (__is_same(PixT, __half)) {
                const float2 f0 = __half22float2(__builtin_bit_cast(__half2, w0));
                const float2 f1 = __half22float2(__builtin_bit_cast(__half2, w1));
                D[0] = {f0.x, f0.y};
                D[1] = {f1.x, f1.y};
            } else if constexpr (__is_same(PixT, int16_t)) {
                D[0] = i16x2_to_float(w0);
                D[1] = i16x2_to_float(w1);
            } else {
                D[0] = {__uint_as_float(w0 << 16), __uint_as_float(w0 & 0xffff0000u)};
                D[1] = {__uint_as_float(w1 << 16), __uint_as_float(w1 & 0xffff0000u)};
            }
        }
    } else if constexpr (LAYOUT == 2 && C % 4 == 0 && __is_same(PixT, int16_t)) {
        // a multiple of four int16 channels side by side (several realisations interleaved): 16-byte loads
#pragma unroll
        for (int c = 0; c < C; c += 4) {
            const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + (uint32_t)(c * 4), 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) D[c + e] = i16x2_to_float((uint32_t)q[e]);
        }
    } else if constexpr (LAYOUT == 2 && C % 2 == 0 && sizeof(PixT) == 4) {
        // an even number of FP32 channels side by side (several realisations interleaved): 16-byte loads
#pragma unroll
        for (int c = 0; c < C; c += 2) {
            const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + (uint32_t)(c * 8), 0));
            D[c] = {q.x, q.y};
            D[c + 1] = {q.z, q.w};
        }
    } else if constexpr (LAYOUT == 2 && C == 3 && sizeof(PixT) == 4) {
        // A and E with one 16-byte load, T with one 8-byte load (24-byte cells, 8-byte aligned)
        const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
        const float2 t = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff + 16u, 0));
        D[0] = {q.x, q.y};
        D[1] = {q.z, q.w};
        D[2] = {t.x, t.y};
    } else if constexpr (LAYOUT == 2) {
        // one or three channels side by side: one load per channel at the pixel size apart
#pragma unroll
        for (int c = 0; c < C; ++c) D[c] = buf_load<PixT>(r, voff, soff + (uint32_t)(c * 2 * sizeof(PixT)));
    } else {
#pragma unroll
        for (int c = 0; c < C; ++c) D[c] = buf_load<PixT>(r, voff, soff + (uint32_t)c * chan);
    }
}

// Tranche sums of the WAVE schedule.  A bin on the wave's band [jA, jB] adds its exact
// weighted value g directly: P_c += conj(D_c) g, Q += |g|^2.  Every other bin takes the
// asymptotic form g = i Q w (E0 / (x - j) - E1 / (x - j + beta)), written with
//   r = w / ((x - j)(x - j + beta)),  b = (x - j) r = w / (x - j + beta)
// as g = beta r E0' + b Delta',  E0' = i Q E0,  Delta' = i Q (E0 - E1).
// The bin then adds only real multiples of conj(D_c) and the products r^2, b^2, r b; the
// tranche constants are applied once at the end (finish).  beta r carries the difference of
// the two edge terms without cancellation, and outside the band the two parts of g are
// never close to opposite, so |g|^2 summed from the three products keeps FP32 precision.
template <int C, class R>
struct BinSums {
    cx<R> P[C];          // band bins: sum conj(D_c) g
    R Q;                 // band bins: sum |g|^2
    cx<R> Ar[C], Ab[C];  // asymptotic bins: sum r conj(D_c), sum b conj(D_c)
    R Srr, Sbb, Srb;     // asymptotic bins: sum r^2, b^2, r b

    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int c = 0; c < C; ++c) P[c] = Ar[c] = Ab[c] = {(R)0, (R)0};
        Q = Srr = Sbb = Srb = (R)0;
    }

    // P_c and Q of the whole tranche
    __device__ __forceinline__ void finish(const TrancheSpec<R> &ts, cx<R> (&Pc)[C], R &Qc) const {
#pragma clang fp contract(fast)
        const R qb = ts.Q * ts.beta;
        const cx<R> e0 = {-qb * ts.E0.im, qb * ts.E0.re};  // beta E0'
        const cx<R> dl = {-ts.Q * (ts.E0.im - ts.E1.im), ts.Q * (ts.E0.re - ts.E1.re)};
#pragma unroll
        for (int c = 0; c < C; ++c) Pc[c] = cadd(P[c], cadd(cmul(e0, Ar[c]), cmul(dl, Ab[c])));
        const R n0 = e0.re * e0.re + e0.im * e0.im;
        const R n1 = dl.re * dl.re + dl.im * dl.im;
        const R x01 = e0.re * dl.re + e0.im * dl.im;
        Qc = Q + n0 * Srr + n1 * Sbb + (R)2 * x01 * Srb;
    }
};

template <int C, class R, class PixT, int FR = kFresnelPaper>
__device__ __forceinline__ void bin_accumulate(const TrancheSpec<R> &ts, int j, R xj, R w, int jA, int jB,
                                               const cx<typename PixTraits<PixT>::R> (&Dl)[C],
                                               const float *__restrict__ sc_bin, int KP, BinSums<C, R> &acc) {
#pragma clang fp contract(fast)
    cx<R> D[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        D[c] = {(R)Dl[c].re, (R)Dl[c].im};
        if constexpr (PixTraits<PixT>::scaled) {
            const R s = (R)sc_bin[c * KP];
            D[c].re *= s;
            D[c].im *= s;
        }
    }
    if (j >= jA && j <= jB) {
        const cx<R> h = bin_full<R, FR>(ts, xj, j);
        const cx<R> g = {h.re * w, h.im * w};
        acc.Q += g.re * g.re;
        acc.Q += g.im * g.im;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            // conj(D) g accumulated as four separate multiply-adds
            acc.P[c].re += D[c].re * g.re;
            acc.P[c].re += D[c].im * g.im;
            acc.P[c].im += D[c].re * g.im;
            acc.P[c].im -= D[c].im * g.re;
        }
    } else {
        const R xj1 = xj + ts.beta;
        R r;
        if constexpr (sizeof(R) == 4)
            r = rcp(xj * xj1) * w;
        else
            r = w / (xj * xj1);
        const R b = xj * r;
        acc.Srr += r * r;
        acc.Sbb += b * b;
        acc.Srb += r * b;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc.Ar[c].re += r * D[c].re;
            acc.Ar[c].im -= r * D[c].im;
            acc.Ab[c].re += b * D[c].re;
            acc.Ab[c].im -= b * D[c].im;
        }
    }
}

// Bins of one tranche for the WAVE schedule, fully unrolled (bin offsets are immediates) in
// groups of three whose pixel loads are all issued before the group's first bin is evaluated
// (a load consumed inside the band/asymptotic branch is otherwise waited for at once).  Each
// bin's pixel row is a scalar offset from the lane's row of bin kc - 10, and the weight table
// is padded with zeros so bins outside [1, M/2 - 1] contribute nothing.  The band-end rule keeps kc + 10 <= M/2, so every row
// read lies in the store; a lane with kc < 10 would need a row below 0, and a wave holding
// such a lane takes wave_tranche_bins_low instead.  The exact Fresnel form is used only for
// the bins [jA, jB] where some lane of the wave may need it (a wave-uniform choice).
template <int C, class R, class PixT, int LAYOUT, bool RHO, int FR = kFresnelPaper>
__device__ __forceinline__ void wave_tranche_bins(const TrancheSpec<R> &ts, int kc, int m, int Nt, int K,
                                                  __amdgpu_buffer_rsrc_t rsrc, __amdgpu_buffer_rsrc_t rho_rsrc,
                                                  const R *__restrict__ u_pad, const float *__restrict__ sc_pad,
                                                  int jA, int jB, cx<R> (&P)[C], R &Q) {
    constexpr uint32_t B = sizeof(PixT) == 8 ? 16u : (sizeof(PixT) == 4 ? 8u : 4u);
    constexpr uint32_t BP = LAYOUT == 2 ? (uint32_t)C * B : B;  // bytes per (bin, tranche) cell
    constexpr int NB = 2 * kHalfBins + 1, G = 3;
    static_assert(NB % G == 0, "bin groups must tile the window");
    const uint32_t voff = (uint32_t)((kc - kHalfBins) * Nt + m) * BP;
    const uint32_t row = (uint32_t)Nt * BP, chan = (uint32_t)K * row;
    const uint32_t voff_rho = (uint32_t)((kc - kHalfBins) * Nt + m) * 4u, row_rho = (uint32_t)Nt * 4u;
    const int KP = K + 2 * kHalfBins;
    const R *uk = u_pad + kc;  // uk[jj] = u_pad[kc + jj] = u_{kc + jj - 10}
    const float *sk = sc_pad + kc;
    BinSums<C, R> acc;
    acc.zero();
#pragma unroll
    for (int j0 = 0; j0 < NB; j0 += G) {
        cx<typename PixTraits<PixT>::R> Dl[G][C];
        float rh[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            bin_pixels<C, PixT, LAYOUT>(rsrc, voff, (uint32_t)(j0 + u) * row, chan, Dl[u]);
            if constexpr (RHO)
                rh[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                      rho_rsrc, voff_rho, (uint32_t)(j0 + u) * row_rho, 0));
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int j = j0 + u - kHalfBins;
            R w = uk[j0 + u];
            if constexpr (RHO) w *= (R)rh[u];
            bin_accumulate<C, R, PixT, FR>(ts, j, ts.x - (R)j, w, jA, jB, Dl[u], sk + j0 + u, KP, acc);
        }
    }
    acc.finish(ts, P, Q);
}

// As wave_tranche_bins for a wave with some lane below bin 10: each bin's row is a per-lane
// offset, clamped at row 0 (rows below 0 have weight 0, so the clamped load adds nothing).
// Same arithmetic in the same order, so a lane's result does not depend on its wave.
template <int C, class R, class PixT, int LAYOUT, bool RHO, int FR = kFresnelPaper>
__device__ __forceinline__ void wave_tranche_bins_low(const TrancheSpec<R> &ts, int kc, int m, int Nt, int K,
                                                   __amdgpu_buffer_rsrc_t rsrc, __amdgpu_buffer_rsrc_t rho_rsrc,
                                                   const R *__restrict__ u_pad, const float *__restrict__ sc_pad,
                                                   int jA, int jB, cx<R> (&P)[C], R &Q) {
    constexpr uint32_t B = sizeof(PixT) == 8 ? 16u : (sizeof(PixT) == 4 ? 8u : 4u);
    constexpr uint32_t BP = LAYOUT == 2 ? (uint32_t)C * B : B;
    const uint32_t chan = (uint32_t)K * (uint32_t)Nt * BP;
    const int KP = K + 2 * kHalfBins;
    const R *uk = u_pad + kc;
    const float *sk = sc_pad + kc;
    BinSums<C, R> acc;
    acc.zero();
#pragma unroll 1
    for (int jj = 0; jj < 2 * kHalfBins + 1; ++jj) {
        const int j = jj - kHalfBins;
        const int k = max(kc + j, 0);
        cx<typename PixTraits<PixT>::R> Dl[C];
        bin_pixels<C, PixT, LAYOUT>(rsrc, (uint32_t)(k * Nt + m) * BP, 0u, chan, Dl);
        R w = uk[jj];
        if constexpr (RHO)
            w *= (R)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rho_rsrc, (uint32_t)(k * Nt + m) * 4u, 0u, 0));
        bin_accumulate<C, R, PixT, FR>(ts, j, ts.x - (R)j, w, jA, jB, Dl, sk + jj, KP, acc);
    }
    acc.finish(ts, P, Q);
}

// Per-template constants are the same in every lane of a wave; stating that with
// readfirstlane lets the compiler keep them in scalar registers instead of 64-lane
// vector registers, which the tranche loop needs for occupancy.
__device__ __forceinline__ double wave_uniform(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float wave_uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
}

__device__ __forceinline__ void wave_uniform(Track &T) {
    T.eta = wave_uniform(T.eta);
    T.M = wave_uniform(T.M);
    T.c8 = wave_uniform(T.c8);
    T.a2 = wave_uniform(T.a2);
    T.a3 = wave_uniform(T.a3);
    T.a4 = wave_uniform(T.a4);
    T.b2 = wave_uniform(T.b2);
    T.b3 = wave_uniform(T.b3);
    T.b4 = wave_uniform(T.b4);
    T.tc = wave_uniform(T.tc);
    T.th0 = wave_uniform(T.th0);
    T.M5 = wave_uniform(T.M5);
    T.M40 = wave_uniform(T.M40);
    T.r5M = wave_uniform(T.r5M);
    T.rc8 = wave_uniform(T.rc8);
    T.r40M = wave_uniform(T.r40M);
    T.reta = wave_uniform(T.reta);
}

template <class R>
__device__ __forceinline__ void wave_uniform(Sky<R> &S) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        S.k[q] = wave_uniform(S.k[q]);
        S.u[q] = wave_uniform(S.u[q]);
        S.v[q] = wave_uniform(S.v[q]);
        S.kd[q] = wave_uniform(S.kd[q]);
    }
    S.q = wave_uniform(S.q);
}

// ------------------------------------------------------------------ THREAD schedule
// The body of the thread-per-template kernels (k_stat_thread; the accurate-Fresnel variant).
template <int C, class R, class PixT, int LAYOUT, bool RHO, int FR, bool LK = false>
__device__ __forceinline__ void stat_thread_body(const StatArgs &a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    int64_t i = a.order ? (int64_t)a.order[t] : t;
    if (i < 0 || i >= a.n) return;  // malformed processing order: skip rather than fault
    const int ns = a.nseg[i];
    const int64_t off = a.seg_offset[i];
    SegAcc<double> acc{0, 0, 0, 0, 0, false};
    int flag = 0;
    if (!params_valid(a.mc[i], a.eta[i], a.f0[i], a.ct[i], a.ci[i])) {
        flag = kFlagInvalid;
        close_segments(acc, ns, off, a.seg_terms, a.seg_zn, true);
        a.stat[i] = 0.0;
        a.flags[i] = flag;
        if (a.n_active) a.n_active[i] = 0;
        return;
    }
    Track T;
    track_init(T, a.mc[i], a.eta[i], a.f0[i]);
    Sky<R> S;
    sky_init(S, a.ct[i], a.phi[i], a.psi[i], a.ci[i]);
    const GeoView gv = geo_view(a.geo, a.geo32, a.Nt, LK ? a.links : nullptr, LK ? a.tdi2 : 0);
    const double u_mul = a.u_scale[0];
    int m = 0, n_act = 0;
    for (; m < a.Nt; ++m) {
        double tm = (double)m * a.dT, Phi, f, fdot;
        int code = track_step(T, tm, a.dT, a.df, a.fnyq, Phi, f, fdot);
        if (code) {
            flag |= code;
            break;
        }
        int sg = (int)(((int64_t)m * ns) / a.Nt);
        close_segments(acc, sg, off, a.seg_terms, a.seg_zn, true);
        double wmd = a.tranche_w[m];
        if (wmd == 0.0) continue;
        ++n_act;
        TrancheSpec<R> ts;
        int kc = tranche_setup(ts, Phi, f, fdot, a.dT);
        cx<R> P[C];
        R Q;
        tranche_bins<C, R, PixT, LAYOUT, double, RHO, FR>(a, ts, kc, m, a.inv_asd, u_mul, a.layer_scale, P, Q);
        R zr, zi, nn;
        tranche_combine<C, R, LK>(S, gv, m, f, (R)wmd, P, Q, zr, zi, nn);
        acc.zr += zr;
        acc.zi += zi;
        acc.N += nn;
    }
    if (m == 0) flag |= kFlagEmpty;
    close_segments(acc, ns, off, a.seg_terms, a.seg_zn, true);
    if (!acc.any && m > 0) flag |= kFlagAllExcluded;
    a.stat[i] = acc.total;
    a.flags[i] = flag;
    if (a.n_active) a.n_active[i] = n_act;
}

// The body of the wave-per-template kernels (k_stat_wave; the accurate-Fresnel variant, which takes the
// general form on all 21 bins; the unequal-arm variant, LK).
template <int C, class R, class PixT, int LAYOUT, bool RHO, int FR, bool LK = false>
__device__ __forceinline__ void stat_wave_body(const StatArgs &a) {
    // Zero-padded template weights u_pad[k + 10] = u_k for 1 <= k <= M/2 - 1 (else 0), and
    // the 16-bit layer scales, staged in LDS once per block.
    extern __shared__ unsigned char smem_raw[];
    const int KP = a.K + 2 * kHalfBins;
    R *u_pad = reinterpret_cast<R *>(smem_raw);
    float *sc_pad = reinterpret_cast<float *>(smem_raw + sizeof(R) * KP);
    const double u_mul = a.u_scale[0];
    const int kmax = a.M / 2 - 1;
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
        const int k = q - kHalfBins;
        u_pad[q] = (k >= 1 && k <= kmax) ? (R)(a.inv_asd[k] * u_mul) : (R)0;
    }
    if constexpr (PixTraits<PixT>::scaled)
        for (int q = threadIdx.x; q < C * KP; q += blockDim.x) {
            const int c = q / KP, k = q % KP - kHalfBins;
            sc_pad[q] = (k >= 0 && k < a.K) ? a.layer_scale[c * a.K + k] : 0.0f;
        }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rsrc = pix_rsrc(a.pix, a.pix_bytes);
    const __amdgpu_buffer_rsrc_t rho_rsrc = pix_rsrc(RHO ? a.rho : a.pix, RHO ? a.rho_bytes : 0u);
    const GeoView gv = geo_view(a.geo, a.geo32, a.Nt, LK ? a.links : nullptr, LK ? a.tdi2 : 0);

    const int lane = threadIdx.x & 63;
    for (;;) {
        // Work fetch in converged code: every lane joins one atomic on a uniform address
        // (lane 0 adds 1, the others 0), which the compiler turns into a single atomic per
        // wave, and readfirstlane makes the item a wave-uniform scalar, so no cross-lane
        // broadcast depends on reconvergence after a lane-0-only branch.
        const uint32_t mine = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(mine);
        if (item >= a.n) break;
        const int64_t i = a.order ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[item]) : item;
        if (i < 0 || i >= a.n) continue;  // malformed processing order: skip rather than fault
        const int ns = a.nseg[i];
        const int64_t off = a.seg_offset[i];
        SegAcc<double> acc{0, 0, 0, 0, 0, false};
        int flag = 0;
        const bool writer = lane == 0;
        if (!params_valid(a.mc[i], a.eta[i], a.f0[i], a.ct[i], a.ci[i])) {
            close_segments(acc, ns, off, a.seg_terms, a.seg_zn, writer);
            if (writer) {
                a.stat[i] = 0.0;
                a.flags[i] = kFlagInvalid;
                if (a.n_active) a.n_active[i] = 0;
            }
            continue;
        }
        Track T;
        track_init(T, a.mc[i], a.eta[i], a.f0[i]);
        wave_uniform(T);
        Sky<R> S;
        sky_init(S, a.ct[i], a.phi[i], a.psi[i], a.ci[i]);
        wave_uniform(S);
        int m_end = a.Nt, n_act = 0;
        SegWalk sw;
        sw.init(a.Nt, ns);
        // The track of a chunk is evaluated during the previous chunk, in the same block as that chunk's
        // response, so the dependent FP64 chain and the FP32 response fill each other's issue gaps.
        double Phi, f, fdot;
        int code = track_step_lanes(T, (double)(lane < a.Nt ? lane : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi, f,
                                    fdot);
        code = lane < a.Nt ? code : 0;
        for (int m0 = 0; m0 < m_end; m0 += 64) {
            const int m = m0 + lane;
            const bool inr = m < a.Nt;
            const double wm_raw = inr ? a.tranche_w[m] : 0.0;
            const uint64_t viol = __ballot(code != 0);
            int lim = a.Nt;
            if (viol) {
                const int first = __builtin_amdgcn_readfirstlane(__ffsll((unsigned long long)viol) - 1);
                lim = m0 + first;
                flag |= __builtin_amdgcn_readlane(code, first);
                m_end = lim;
            }
            const bool active = inr && m < lim;
            const double wmd = active ? wm_raw : 0.0;
            const bool work = active && wmd != 0.0;
            n_act += __popcll(__ballot(work));
            TrancheSpec<R> ts;
            int kc = 0;
            int nlo = INT_MIN, hi = INT_MIN;  // -(first) and last bin that is not asymptotic-only
            if (work) {
                kc = tranche_setup(ts, Phi, f, fdot, a.dT);
                nlo = -ts.j0lo;
                hi = ts.j1hi;
            }
            // The wave takes the general form on the union [jA, jB] of the lanes' such bins (on all bins in the
            // accurate Fresnel mode, which has no asymptotic-only form).
            int jA = -kHalfBins, jB = kHalfBins;
            if constexpr (FR == kFresnelPaper) {
                wave_max2_i32(nlo, hi);
                jA = -nlo;
                jB = hi;
            }
            R zr = 0, zi = 0, nn = 0;
            const bool low = __ballot(work && kc < kHalfBins) != 0;
            cx<R> P[C];
            R Q = 0;
            if (work) {
                if (low)
                    wave_tranche_bins_low<C, R, PixT, LAYOUT, RHO, FR>(ts, kc, m, a.Nt, a.K, rsrc, rho_rsrc, u_pad, sc_pad,
                                                                   jA, jB, P, Q);
                else
                    wave_tranche_bins<C, R, PixT, LAYOUT, RHO, FR>(ts, kc, m, a.Nt, a.K, rsrc, rho_rsrc, u_pad, sc_pad,
                                                               jA, jB, P, Q);
            }
            // this chunk's response and the next chunk's track, for every lane (values of lanes without work
            // are not used; the geometry row is clamped into the table)
            cx<R> Tc[C];
            tranche_transfer<C, R, LK>(S, gv, inr ? m : a.Nt - 1, f, Tc);
            {
                const int mn = m + 64;
                int cn = track_step_lanes(T, (double)(mn < a.Nt ? mn : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi, f,
                                          fdot);
                code = mn < a.Nt ? cn : 0;
            }
            if (work) tranche_sums<C, R>(Tc, (R)wmd, P, Q, zr, zi, nn);
            // segmented reduction over the lanes of this chunk
            const int last = min(min(m0 + 63, lim - 1), a.Nt - 1);
            if (last >= m0) {
                while (sw.hi <= m0) sw.step();
                for (;;) {
                    const bool mine = active && m >= sw.lo && m < sw.hi;
                    R vr = mine ? zr : (R)0, vi = mine ? zi : (R)0, vn = mine ? nn : (R)0;
                    wave_sum3<R>(vr, vi, vn);
                    close_segments(acc, sw.s, off, a.seg_terms, a.seg_zn, writer);
                    acc.zr += (double)vr;
                    acc.zi += (double)vi;
                    acc.N += (double)vn;
                    if (sw.hi > last) break;
                    sw.step();
                }
            }
            if (viol) break;
        }
        if (m_end == 0) flag |= kFlagEmpty;
        close_segments(acc, ns, off, a.seg_terms, a.seg_zn, writer);
        if (!acc.any && m_end > 0) flag |= kFlagAllExcluded;
        if (writer) {
            a.stat[i] = acc.total;
            a.flags[i] = flag;
            if (a.n_active) a.n_active[i] = n_act;
        }
    }
}

inline StatArgs make_args(const StatLaunch &L) {
    StatArgs a;
    a.M = L.M;
    a.K = L.M / 2 + 1;
    a.Nt = L.Nt;
    a.C = L.C;
    a.dt = L.dt;
    a.dT = (double)L.M * L.dt;
    a.df = 1.0 / a.dT;
    a.fnyq = 0.5 / L.dt;
    a.pix = L.pix;
    {
        const size_t pb = L.pix_dtype == 0 ? 16 : (L.pix_dtype == 1 ? 8 : 4);
        const size_t tot = pb * (size_t)L.C * (size_t)(L.M / 2 + 1) * (size_t)L.Nt;
        a.pix_bytes = tot > 0xffffffffull ? 0xffffffffu : (uint32_t)tot;
    }
    a.layer_scale = L.layer_scale;
    a.inv_asd = L.inv_asd;
    a.tranche_w = L.tranche_w;
    a.geo = L.geo;
    a.geo32 = geo32_of(L.geo, L.Nt);
    a.u_scale = L.u_scale;
    a.rho = L.rho;
    a.links = L.links;
    a.tdi2 = L.tdi2;
    {
        const uint64_t rb = (uint64_t)a.K * (uint64_t)a.Nt * 4u;
        a.rho_bytes = L.rho ? (rb > 0xffffffffull ? 0xffffffffu : (uint32_t)rb) : 0u;
    }
    a.n = L.n;
    a.mc = L.mc;
    a.eta = L.eta;
    a.f0 = L.f0;
    a.ct = L.ct;
    a.phi = L.phi;
    a.psi = L.psi;
    a.ci = L.ci;
    a.nseg = L.nseg;
    a.seg_offset = L.seg_offset;
    a.order = L.order;
    a.seg_terms = L.seg_terms;
    a.stat = L.stat;
    a.seg_zn = L.seg_zn;
    a.flags = L.flags;
    a.n_active = L.n_active;
    a.counter = L.counter;
    a.real_stride = 0;
    a.seg_stride = 0;
    a.rho0 = 0;
    return a;
}

}  // namespace tfsc
