// The statistic for multi-harmonic templates (paper Sec. "Outlook": the waveform quantities {A, f, fdot, phi}
// are computed for each harmonic and the Fresnel expressions applied to each).
//
// Harmonic h of the orbital phase has phase (h/2) Phi, frequency (h/2) f and chirp (h/2) fdot, with
// (Phi, f, fdot) the dominant harmonic's FP64 track, amplitude a_h A with A = f^(2/3) and a_h a complex
// factor per template, the dominant harmonic's polarisation pattern and its own TDI transfer T_c(t_m, f_h).
// In each tranche harmonic h fills its own 21 bins around k_c,h = ceil(f_h dT); the template pixel of a bin
// is the sum over the harmonics whose window holds it.  So, per tranche,
//   z = sum_h sum_c a_h T_c,h P_c,h,   N = sum_h sum_c |a_h T_c,h|^2 Q_h + 2 Re sum_{h<h'} K_hh' X_hh',
// with P, Q each harmonic's own 21-bin sums (the single-harmonic kernel's), K_hh' = sum_c a_h T_c,h
// conj(a_h' T_c,h') and X_hh' = sum over the bins both windows hold of g_h conj(g_h') (g the weighted bin
// values).  Windows overlap only at low frequency (orbital frequency below 21 bins); a lane whose tranche
// has such a pair evaluates X on the shared bins by itself.
//
// The track ends where the single-harmonic rule ends it for the merger, and where the highest harmonic of
// the set violates the band or compactness condition.  Wave schedule (one 64-lane wavefront per template,
// lanes over tranches), LAYER_MAJOR or LAYER_MAJOR_CI stores, FP64 or FP32 pixels with the same arithmetic,
// separable PSD, the paper's Fresnel forms.
#include "tfsc_stat_common.hpp"

namespace tfsc {

struct HarmArgs {
    int n;                 // harmonics in the set, 1..kMaxHarmonics
    int h[kMaxHarmonics];  // harmonic numbers of the orbital phase, 1..8
    double smax;           // the largest h / 2
    const double *amp;     // [templates][n][2] complex factors a_h
};

__device__ __forceinline__ int track_step_harm(const Track &T, double tm, double dT, double df, double fnyq,
                                               double smax, double &Phi, double &f, double &fdot) {
    if (tm + dT >= T.tc) return kFlagMergeEnd;
    track_at(T, tm, Phi, f, fdot);
    if ((smax * (f + fdot * dT) >= fnyq - 11.0 * df) || (smax * fdot * dT > 10.0 * df)) return kFlagBandEnd;
    return 0;
}

template <int C, class R>
__device__ __forceinline__ void harmonic_response(const Sky<R> &S, const GeoView &gv, int m, double fh, cx<R> amp,
                                                  cx<R> (&Tp)[C]) {
    cx<R> TA, TE, TT;
    transfer_ae<R, (C == 3)>(S, gv, m, fh, TA, TE, &TT);
    Tp[0] = cmul(amp, TA);
    if constexpr (C >= 2) Tp[1] = cmul(amp, TE);
    if constexpr (C == 3) Tp[2] = cmul(amp, TT);
}

template <class R>
__device__ __forceinline__ cx<R> harmonic_amp(const HarmArgs &hm, int64_t i, int q) {
    const double *p = hm.amp + 2 * ((size_t)i * hm.n + q);
    return {(R)p[0], (R)p[1]};
}

// 2 Re(K X) for harmonics q < r of one lane's tranche whose windows share bins.
template <int C, class R>
__device__ __noinline__ R harmonic_cross(const HarmArgs &hm, int64_t i, int q, int r, double Phi, double f,
                                         double fdot, double dT, const R *__restrict__ u_pad, const Sky<R> &S,
                                         const GeoView &gv, int m) {
#pragma clang fp contract(fast)
    const double sq = 0.5 * (double)hm.h[q], sr = 0.5 * (double)hm.h[r];
    TrancheSpec<R> tq, tr;
    const int kq = tranche_setup(tq, sq * Phi, sq * f, sq * fdot, dT, f);
    const int kr = tranche_setup(tr, sr * Phi, sr * f, sr * fdot, dT, f);
    const int lo = max(kq, kr) - kHalfBins, hi = min(kq, kr) + kHalfBins;
    cx<R> X = {(R)0, (R)0};
    for (int k = lo; k <= hi; ++k) {
        const R w = u_pad[k + kHalfBins];  // 0 outside bins 1 .. M/2 - 1
        const cx<R> gq = tranche_bin_weighted(tq, k - kq, w);
        const cx<R> gr = tranche_bin_weighted(tr, k - kr, w);
        X.re += gq.re * gr.re + gq.im * gr.im;
        X.im += gq.im * gr.re - gq.re * gr.im;
    }
    cx<R> Tq[C], Tr[C];
    harmonic_response<C, R>(S, gv, m, sq * f, harmonic_amp<R>(hm, i, q), Tq);
    harmonic_response<C, R>(S, gv, m, sr * f, harmonic_amp<R>(hm, i, r), Tr);
    cx<R> K = {(R)0, (R)0};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        K.re += Tq[c].re * Tr[c].re + Tq[c].im * Tr[c].im;
        K.im += Tq[c].im * Tr[c].re - Tq[c].re * Tr[c].im;
    }
    return (R)2 * (K.re * X.re - K.im * X.im);
}

template <int C, class R, class PixT, int LAYOUT>
__global__ __launch_bounds__(256, 2) void k_stat_wave_harm(StatArgs a, HarmArgs hm) {
    extern __shared__ unsigned char smem_raw[];
    const int KP = a.K + 2 * kHalfBins;
    R *u_pad = reinterpret_cast<R *>(smem_raw);
    const double u_mul = a.u_scale[0];
    const int kmax = a.M / 2 - 1;
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
        const int k = q - kHalfBins;
        u_pad[q] = (k >= 1 && k <= kmax) ? (R)(a.inv_asd[k] * u_mul) : (R)0;
    }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rsrc = pix_rsrc(a.pix, a.pix_bytes);
    const GeoView gv = geo_view(a.geo, a.geo32, a.Nt);
    const int lane = threadIdx.x & 63;
    for (;;) {
        const uint32_t mine = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(mine);
        if (item >= a.n) break;
        const int64_t i = a.order ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[item]) : item;
        if (i < 0 || i >= a.n) continue;
        const int ns = a.nseg[i];
        const int64_t off = a.seg_offset[i];
        SegAcc<double> acc{0, 0, 0, 0, 0, false};
        int flag = 0;
        const bool writer = lane == 0;
        const double mci = a.mc[i];
        if (!params_valid(mci, a.eta[i], a.f0[i], a.ct[i], a.ci[i])) {
            close_segments(acc, ns, off, a.seg_terms, a.seg_zn, writer);
            if (writer) {
                a.stat[i] = 0.0;
                a.flags[i] = kFlagInvalid;
                if (a.n_active) a.n_active[i] = 0;
            }
            continue;
        }
        Track T;
        track_init(T, mci, a.eta[i], a.f0[i]);
        wave_uniform(T);
        Sky<R> S;
        sky_init(S, a.ct[i], a.phi[i], a.psi[i], a.ci[i]);
        wave_uniform(S);
        int m_end = a.Nt, n_act = 0;
        SegWalk sw;
        sw.init(a.Nt, ns);
        for (int m0 = 0; m0 < m_end; m0 += 64) {
            const int m = m0 + lane;
            const bool inr = m < a.Nt;
            const double wm_raw = inr ? a.tranche_w[m] : 0.0;
            double Phi = 0.0, f = 0.0, fdot = 0.0;
            int code = inr ? track_step_harm(T, (double)m * a.dT, a.dT, a.df, a.fnyq, hm.smax, Phi, f, fdot) : 0;
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
            cx<R> z = {(R)0, (R)0};
            R nn = 0;
            uint32_t kpack0 = 0, kpack1 = 0;  // k_c of the harmonics, 16 bits each
#pragma unroll 1
            for (int q = 0; q < hm.n; ++q) {
                const double s = 0.5 * (double)hm.h[q];
                TrancheSpec<R> ts;
                int kc = 0;
                int nlo = INT_MIN, hi = INT_MIN;
                if (work) {
                    kc = tranche_setup(ts, s * Phi, s * f, s * fdot, a.dT, f);
                    nlo = -ts.j0lo;
                    hi = ts.j1hi;
                }
                wave_max2_i32(nlo, hi);
                const int jA = -nlo, jB = hi;
                const bool low = __ballot(work && kc < kHalfBins) != 0;
                const uint32_t kbits = (uint32_t)kc & 0xffffu;
                if (q == 0) kpack0 = kbits;
                else if (q == 1) kpack0 |= kbits << 16;
                else if (q == 2) kpack1 = kbits;
                else kpack1 |= kbits << 16;
                if (work) {
                    cx<R> P[C];
                    R Q;
                    if (low)
                        wave_tranche_bins_low<C, R, PixT, LAYOUT, false>(ts, kc, m, a.Nt, a.K, rsrc, rsrc, u_pad,
                                                                         nullptr, jA, jB, P, Q);
                    else
                        wave_tranche_bins<C, R, PixT, LAYOUT, false>(ts, kc, m, a.Nt, a.K, rsrc, rsrc, u_pad,
                                                                     nullptr, jA, jB, P, Q);
                    cx<R> Tp[C];
                    harmonic_response<C, R>(S, gv, m, s * f, harmonic_amp<R>(hm, i, q), Tp);
                    R tt = 0;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        z = cadd(z, cmul(Tp[c], P[c]));
                        tt += Tp[c].re * Tp[c].re + Tp[c].im * Tp[c].im;
                    }
                    nn += tt * Q;
                }
            }
            if (work && hm.n > 1) {
                for (int q = 0; q < hm.n; ++q)
                    for (int r = q + 1; r < hm.n; ++r) {
                        const uint32_t wq = q < 2 ? kpack0 : kpack1, wr = r < 2 ? kpack0 : kpack1;
                        const int kq = (int)((wq >> (16 * (q & 1))) & 0xffffu);
                        const int kr = (int)((wr >> (16 * (r & 1))) & 0xffffu);
                        if (abs(kq - kr) <= 2 * kHalfBins)
                            nn += harmonic_cross<C, R>(hm, i, q, r, Phi, f, fdot, a.dT, u_pad, S, gv, m);
                    }
            }
            const R wmr = (R)wmd;
            const R zr = wmr * z.re, zi = wmr * z.im;
            nn = wmr * wmr * nn;
            // segmented reduction over the lanes of this chunk
            const int last = min(min(m0 + 63, lim - 1), a.Nt - 1);
            if (last >= m0) {
                while (sw.hi <= m0) sw.step();
                for (;;) {
                    const bool mine2 = active && m >= sw.lo && m < sw.hi;
                    R vr = mine2 ? zr : (R)0, vi = mine2 ? zi : (R)0, vn = mine2 ? nn : (R)0;
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

template <int C, class R, class PixT>
static hipError_t launch_harm_t(const StatLaunch &L, const StatArgs &a, const HarmArgs &hm, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, a.counter, 1);
    const size_t shmem = sizeof(R) * ((size_t)a.K + 2 * kHalfBins);
    if (L.layout == 2)
        hipLaunchKernelGGL((k_stat_wave_harm<C, R, PixT, 2>), dim3(L.n_groups), dim3(64 * L.block_waves), shmem, st,
                           a, hm);
    else
        hipLaunchKernelGGL((k_stat_wave_harm<C, R, PixT, 0>), dim3(L.n_groups), dim3(64 * L.block_waves), shmem, st,
                           a, hm);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_harm_c(const StatLaunch &L, const StatArgs &a, const HarmArgs &hm, hipStream_t st) {
    if (L.precision == 0 && L.pix_dtype == 0) return launch_harm_t<C, double, double>(L, a, hm, st);
    if (L.precision == 1 && L.pix_dtype == 1) return launch_harm_t<C, float, float>(L, a, hm, st);
    return hipErrorInvalidValue;
}

hipError_t launch_statistic_harmonics(const StatLaunch &L, int n_harm, const int *harm, const double *amp,
                                      hipStream_t st) {
    StatArgs a = make_args(L);
    if (L.n == 0) return hipSuccess;
    if (L.rho || L.schedule != 1 || L.layout == 1 || n_harm < 1 || n_harm > kMaxHarmonics) return hipErrorInvalidValue;
    HarmArgs hm;
    hm.n = n_harm;
    int hmax = 0;
    for (int q = 0; q < kMaxHarmonics; ++q) {
        hm.h[q] = q < n_harm ? harm[q] : 0;
        if (q < n_harm && harm[q] > hmax) hmax = harm[q];
    }
    hm.smax = 0.5 * (double)hmax;
    hm.amp = amp;
    if (L.C == 1) return launch_harm_c<1>(L, a, hm, st);
    if (L.C == 3) return launch_harm_c<3>(L, a, hm, st);
    return launch_harm_c<2>(L, a, hm, st);
}

}  // namespace tfsc
