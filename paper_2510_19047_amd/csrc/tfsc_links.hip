// The statistic with a caller's link light times (unequal arms, varying arm lengths and point-ahead light
// times of a numerical orbit; paper Sec. "Outlook"): the default kernels' bodies with the unequal-arm response
// transfer_links in place of the equal-arm one.  Both schedules; FP64 or FP32 pixels with the same
// arithmetic; separable PSD; the paper's Fresnel forms.
#include "tfsc_stat_common.hpp"

namespace tfsc {

template <int C, class R, class PixT, int LAYOUT>
__global__ __launch_bounds__(256) void k_stat_thread_lk(StatArgs a) {
    stat_thread_body<C, R, PixT, LAYOUT, false, kFresnelPaper, true>(a);
}

template <int C, class R, class PixT, int LAYOUT>
__global__ __launch_bounds__(256, 2) void k_stat_wave_lk(StatArgs a) {
    stat_wave_body<C, R, PixT, LAYOUT, false, kFresnelPaper, true>(a);
}

template <int C, class R, class PixT>
static hipError_t launch_lk_t(const StatLaunch &L, const StatArgs &a, hipStream_t st) {
    if (L.schedule == 0) {
        dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
        if (L.layout == 0)
            hipLaunchKernelGGL((k_stat_thread_lk<C, R, PixT, 0>), grid, block, 0, st, a);
        else if (L.layout == 1)
            hipLaunchKernelGGL((k_stat_thread_lk<C, R, PixT, 1>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((k_stat_thread_lk<C, R, PixT, 2>), grid, block, 0, st, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, a.counter, 1);
    const size_t shmem = sizeof(R) * ((size_t)a.K + 2 * kHalfBins);
    if (L.layout == 2)
        hipLaunchKernelGGL((k_stat_wave_lk<C, R, PixT, 2>), dim3(L.n_groups), dim3(64 * L.block_waves), shmem, st, a);
    else
        hipLaunchKernelGGL((k_stat_wave_lk<C, R, PixT, 0>), dim3(L.n_groups), dim3(64 * L.block_waves), shmem, st, a);
    return hipGetLastError();
}

template <int C>
static hipError_t launch_lk_c(const StatLaunch &L, const StatArgs &a, hipStream_t st) {
    if (L.precision == 0 && L.pix_dtype == 0) return launch_lk_t<C, double, double>(L, a, st);
    if (L.precision == 1 && L.pix_dtype == 1) return launch_lk_t<C, float, float>(L, a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_statistic_links(const StatLaunch &L, hipStream_t st) {
    StatArgs a = make_args(L);
    if (L.n == 0) return hipSuccess;
    if (L.rho || !L.links) return hipErrorInvalidValue;
    if (L.C == 1) return launch_lk_c<1>(L, a, st);
    if (L.C == 3) return launch_lk_c<3>(L, a, st);
    return launch_lk_c<2>(L, a, st);
}

}  // namespace tfsc
