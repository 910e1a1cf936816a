// Several noise realisations interleaved in one pixel store (paper Sec. "Results": the background
// comes from many noise-only realisations; Sec. "Hardware acceleration and computational cost":
// large batches per launch).
//
// Layout [K][Nt][NR][C]: each (bin, tranche) cell holds the C channels of each of the NR
// realisations side by side, so the cell is the channel-interleaved cell of one store with NR C
// channels (FP32, or int16 pairs with the NR C channels' layer scales as [NR C][K]).  A template's track, Fresnel bins, response and Q are formed once per tranche; each
// bin's NR C pixels come in wide loads, and the bin sums are those of the single-realisation WAVE
// kernel with the cell's NR C values taken as channels.  Realisation r's tranche sum is
// z_r = w_m sum_c T_c P_{r C + c}; N_n is shared by every realisation.
#include "tfsc_stat_common.hpp"

namespace tfsc {

// Copy one realisation's channel-interleaved store into slot r of an interleaved store (T: one complex
// value, float2 for FP32 or uint32_t for int16 pairs).
template <class T>
__global__ void k_interleave(int64_t cells, int C, int NR, int r, const T *__restrict__ src, T *__restrict__ dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one complex value of the source
    if (e >= cells * C) return;
    const int64_t cell = e / C;
    const int c = (int)(e - cell * C);
    dst[(cell * NR + r) * C + c] = src[e];
}

// The per-layer scales of a 16-bit store: source [C][K] into rows r C .. r C + C - 1 of [NR C][K].
__global__ void k_interleave_scale(int C, int K, int r, const float *__restrict__ src, float *__restrict__ dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < C * K) dst[r * C * K + e] = src[e];
}

hipError_t launch_interleave(int64_t cells, int C, int K, int NR, int r, int elem_bytes, const void *src,
                             const float *src_scale, void *dst, float *dst_scale, hipStream_t st) {
    const int64_t n = cells * C;
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (elem_bytes == 8)
        hipLaunchKernelGGL(k_interleave<float2>, grid, dim3(256), 0, st, cells, C, NR, r,
                           reinterpret_cast<const float2 *>(src), reinterpret_cast<float2 *>(dst));
    else
        hipLaunchKernelGGL(k_interleave<uint32_t>, grid, dim3(256), 0, st, cells, C, NR, r,
                           reinterpret_cast<const uint32_t *>(src), reinterpret_cast<uint32_t *>(dst));
    if (src_scale)
        hipLaunchKernelGGL(k_interleave_scale, dim3((unsigned)((C * K + 255) / 256)), dim3(256), 0, st, C, K, r,
                           src_scale, dst_scale);
    return hipGetLastError();
}

// Segment state for NR realisations: N, cur and any are shared, the rest per realisation.
template <int NR>
struct SegAccRi {
    double zr[NR], zi[NR], total[NR];
    double N;
    int cur;
    bool any;
};

template <int NR>
__device__ __forceinline__ void close_segments_ri(SegAccRi<NR> &acc, int upto, int64_t off, double *seg_terms,
                                                  int64_t seg_stride, bool writer) {
    while (acc.cur < upto) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double v = acc.N > 0.0 ? 2.0 * (acc.zr[r] * acc.zr[r] + acc.zi[r] * acc.zi[r]) / acc.N : 0.0;
            // a plane shorter than the segment layout (a caller error) loses terms instead of overrunning
            if (writer && off + acc.cur < seg_stride) seg_terms[(int64_t)r * seg_stride + off + acc.cur] = v;
            acc.total[r] += v;
            acc.zr[r] = acc.zi[r] = 0.0;
        }
        if (acc.N > 0.0) acc.any = true;
        acc.N = 0.0;
        ++acc.cur;
    }
}

template <int C, int NR, class PixT>
__global__ __launch_bounds__(256, 3) void k_stat_wave_ri(StatArgs a) {
#pragma clang fp contract(fast)
    using R = float;
    constexpr int CC = NR * C;  // values per cell
    extern __shared__ unsigned char smem_raw[];
    const int KP = a.K + 2 * kHalfBins;
    R *u_pad = reinterpret_cast<R *>(smem_raw);
    float *sc_pad = reinterpret_cast<float *>(smem_raw + sizeof(R) * KP);  // int16: the cell's CC layer scales
    const double u_mul = a.u_scale[0];
    const int kmax = a.M / 2 - 1;
    for (int q = threadIdx.x; q < KP; q += blockDim.x) {
        const int k = q - kHalfBins;
        u_pad[q] = (k >= 1 && k <= kmax) ? (R)(a.inv_asd[k] * u_mul) : (R)0;
    }
    if constexpr (PixTraits<PixT>::scaled)
        for (int q = threadIdx.x; q < CC * KP; q += blockDim.x) {
            const int c = q / KP, k = q % KP - kHalfBins;
            sc_pad[q] = (k >= 0 && k < a.K) ? a.layer_scale[c * a.K + k] : 0.0f;
        }
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rsrc = pix_rsrc(a.pix, a.pix_bytes);
    const GeoView gv = geo_view(a.geo, a.geo32, a.Nt);
    const int lane = threadIdx.x & 63;
    const bool writer = lane == 0;
    for (;;) {
        // one atomic per wave on a uniform address, as in k_stat_wave
        const uint32_t mine = atomicAdd(a.counter, lane == 0 ? 1u : 0u);
        const int64_t item = (int64_t)__builtin_amdgcn_readfirstlane(mine);
        if (item >= a.n) break;
        const int64_t i = a.order ? (int64_t)__builtin_amdgcn_readfirstlane(a.order[item]) : item;
        if (i < 0 || i >= a.n) continue;  // malformed processing order: skip rather than fault
        const int ns = a.nseg[i];
        const int64_t off = a.seg_offset[i];
        SegAccRi<NR> acc;
#pragma unroll
        for (int r = 0; r < NR; ++r) acc.zr[r] = acc.zi[r] = acc.total[r] = 0.0;
        acc.N = 0.0;
        acc.cur = 0;
        acc.any = false;
        int flag = 0;
        if (!params_valid(a.mc[i], a.eta[i], a.f0[i], a.ct[i], a.ci[i])) {
            close_segments_ri<NR>(acc, ns, off, a.seg_terms, a.seg_stride, writer);
            if (writer) {
#pragma unroll
                for (int r = 0; r < NR; ++r) a.stat[(int64_t)r * a.n + i] = 0.0;
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
        for (int m0 = 0; m0 < m_end; m0 += 64) {
            const int m = m0 + lane;
            const bool inr = m < a.Nt;
            const double wm_raw = inr ? a.tranche_w[m] : 0.0;
            double Phi, f, fdot;
            int code = track_step_lanes(T, (double)(inr ? m : a.Nt - 1) * a.dT, a.dT, a.df, a.fnyq, Phi, f, fdot);
            code = inr ? code : 0;
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
            int nlo = INT_MIN, hi = INT_MIN;
            if (work) {
                kc = tranche_setup(ts, Phi, f, fdot, a.dT);
                nlo = -ts.j0lo;
                hi = ts.j1hi;
            }
            wave_max2_i32(nlo, hi);
            const int jA = -nlo, jB = hi;
            R zr[NR], zi[NR], nn = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) zr[r] = zi[r] = 0;
            const bool low = __ballot(work && kc < kHalfBins) != 0;
            if (work) {
                cx<R> P[CC];
                R Q;
                if (low)
                    wave_tranche_bins_low<CC, R, PixT, 2, false>(ts, kc, m, a.Nt, a.K, rsrc, rsrc, u_pad, sc_pad,
                                                                 jA, jB, P, Q);
                else
                    wave_tranche_bins<CC, R, PixT, 2, false>(ts, kc, m, a.Nt, a.K, rsrc, rsrc, u_pad, sc_pad, jA,
                                                             jB, P, Q);
                cx<R> TA, TE, TT;
                transfer_ae<R, false>(S, gv, m, f, TA, TE, &TT);
                R tt = TA.re * TA.re + TA.im * TA.im;
                if constexpr (C == 2) tt += TE.re * TE.re + TE.im * TE.im;
                const R wm = (R)wmd;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    cx<R> z = cmul(TA, P[r * C]);
                    if constexpr (C == 2) z = cadd(z, cmul(TE, P[r * C + 1]));
                    zr[r] = wm * z.re;
                    zi[r] = wm * z.im;
                }
                nn = wm * wm * tt * Q;
            }
            // segmented reduction over the lanes of this chunk: N shared, (Re z, Im z) per realisation
            const int last = min(min(m0 + 63, lim - 1), a.Nt - 1);
            if (last >= m0) {
                while (sw.hi <= m0) sw.step();
                for (;;) {
                    const bool mine_seg = active && m >= sw.lo && m < sw.hi;
                    constexpr int NV = 2 * NR + 1, NV3 = (NV + 2) / 3 * 3;
                    R v[NV3];
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        v[2 * r] = mine_seg ? zr[r] : (R)0;
                        v[2 * r + 1] = mine_seg ? zi[r] : (R)0;
                    }
                    v[2 * NR] = mine_seg ? nn : (R)0;
#pragma unroll
                    for (int q = NV; q < NV3; ++q) v[q] = (R)0;
#pragma unroll
                    for (int q = 0; q < NV3; q += 3) wave_sum3<R>(v[q], v[q + 1], v[q + 2]);
                    close_segments_ri<NR>(acc, sw.s, off, a.seg_terms, a.seg_stride, writer);
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        acc.zr[r] += (double)v[2 * r];
                        acc.zi[r] += (double)v[2 * r + 1];
                    }
                    acc.N += (double)v[2 * NR];
                    if (sw.hi > last) break;
                    sw.step();
                }
            }
            if (viol) break;
        }
        if (m_end == 0) flag |= kFlagEmpty;
        close_segments_ri<NR>(acc, ns, off, a.seg_terms, a.seg_stride, writer);
        if (!acc.any && m_end > 0) flag |= kFlagAllExcluded;
        if (writer) {
#pragma unroll
            for (int r = 0; r < NR; ++r) a.stat[(int64_t)r * a.n + i] = acc.total[r];
            a.flags[i] = flag;
            if (a.n_active) a.n_active[i] = n_act;
        }
    }
}

template <int C, int NR, class PixT>
static hipError_t launch_ri_t(const StatArgs &a, int n_groups, int block_waves, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, a.counter, 1);
    const size_t KP = (size_t)a.K + 2 * kHalfBins;
    const size_t shmem = sizeof(float) * KP * (PixTraits<PixT>::scaled ? 1 + NR * C : 1);
    hipLaunchKernelGGL((k_stat_wave_ri<C, NR, PixT>), dim3(n_groups), dim3(64 * block_waves), shmem, st, a);
    return hipGetLastError();
}

template <class PixT>
static hipError_t dispatch_ri(const StatLaunch &L, const StatArgs &a, int g, int bw, hipStream_t st) {
    switch (L.C * 8 + L.n_real) {
        case 8 + 2: return launch_ri_t<1, 2, PixT>(a, g, bw, st);
        case 8 + 4: return launch_ri_t<1, 4, PixT>(a, g, bw, st);
        case 16 + 2: return launch_ri_t<2, 2, PixT>(a, g, bw, st);
        case 16 + 4: return launch_ri_t<2, 4, PixT>(a, g, bw, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_statistic_interleaved(const StatLaunch &L, hipStream_t st) {
    if (L.n == 0) return hipSuccess;
    StatArgs a = make_args(L);
    const uint64_t eb = L.pix_dtype == 4 ? 4ull : 8ull;  // bytes per complex value: int16 pair or FP32
    const uint64_t tot = eb * (uint64_t)L.C * (uint64_t)L.n_real * (uint64_t)(L.M / 2 + 1) * (uint64_t)L.Nt;
    if (tot > 0xffffffffull) return hipErrorInvalidValue;
    a.pix_bytes = (uint32_t)tot;
    a.seg_stride = L.seg_stride;
    const int bw = L.block_waves;
    int64_t groups = (L.n + bw - 1) / bw;
    if (groups > (int64_t)L.n_groups) groups = L.n_groups;
    const int g = (int)groups;
    if (L.pix_dtype == 4) return dispatch_ri<int16_t>(L, a, g, bw, st);
    return dispatch_ri<float>(L, a, g, bw, st);
}

}  // namespace tfsc
