// Evaluation kernels (Section 6): the coverage-weighted k-space average behind the
// baseline reconstructions, and the per-image terms of PSNR on magnitudes.

#include "kcommon.h"

namespace vp {

// Frame slot f of the launch is frame first + f: the average, over the blades
// max(0, first + f - window + 1) .. first + f that measure a sample, of their values
// there (ascending blade order), times 1/n, the unitary scale of the n x n inverse DFT
// that follows. Unmeasured samples are zero. window <= 0 takes every blade up to the frame.
__global__ __launch_bounds__(kThreads) void k_baseline_avg(const uint8_t* __restrict__ mask,
                                                           const float2* __restrict__ y, float2* __restrict__ out,
                                                           int n, int window, int first) {
    const size_t nn = (size_t)n * n;
    const size_t px = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (px >= nn) return;
    const int f = first + (int)blockIdx.y;
    const int lo = window > 0 ? max(0, f - window + 1) : 0;
    float2 acc = make_float2(0.f, 0.f);
    int c = 0;
    for (int b = lo; b <= f; ++b) {
        const size_t i = (size_t)b * nn + px;
        if (mask[i]) {
            acc = cadd(acc, y[i]);
            ++c;
        }
    }
    out[(size_t)blockIdx.y * nn + px] = cscale(acc, 1.0f / ((float)max(c, 1) * (float)n));
}

// One block per image of npx samples: FP64 sum of (|image| - |truth|)^2 and the peak
// |truth|, reduced in a fixed order; terms[3 i + {0, 1, 2}] = mean squared error, peak,
// 10 log10(peak^2 / mse) (+inf for mse = 0).
constexpr int kPsnrThreads = 1024;

__global__ __launch_bounds__(kPsnrThreads) void k_psnr(const float2* __restrict__ img,
                                                       const float2* __restrict__ truth, long long npx,
                                                       double* __restrict__ terms) {
    __shared__ double se[kPsnrThreads];
    __shared__ double pk[kPsnrThreads];
    const size_t off = (size_t)blockIdx.x * (size_t)npx;
    double e = 0.0, m = 0.0;
    for (long long i = threadIdx.x; i < npx; i += kPsnrThreads) {
        const float2 a = img[off + i], t = truth[off + i];
        const double ma = sqrt((double)a.x * a.x + (double)a.y * a.y);
        const double mt = sqrt((double)t.x * t.x + (double)t.y * t.y);
        const double d = ma - mt;
        e = fma(d, d, e);
        m = fmax(m, mt);
    }
    se[threadIdx.x] = e;
    pk[threadIdx.x] = m;
    __syncthreads();
    for (int h = kPsnrThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            se[threadIdx.x] += se[threadIdx.x + h];
            pk[threadIdx.x] = fmax(pk[threadIdx.x], pk[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mse = se[0] / (double)npx, peak = pk[0];
        terms[3 * (size_t)blockIdx.x + 0] = mse;
        terms[3 * (size_t)blockIdx.x + 1] = peak;
        terms[3 * (size_t)blockIdx.x + 2] = mse > 0.0 ? 10.0 * log10(peak * peak / mse) : __builtin_inf();
    }
}

hipError_t launch_baseline_avg(const uint8_t* mask, const float2* y, float2* out, int n, int window, int first,
                               int n_frames, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    const size_t nn = (size_t)n * n;
    const dim3 g((unsigned)((nn + kThreads - 1) / kThreads), (unsigned)n_frames);
    hipLaunchKernelGGL(k_baseline_avg, g, dim3(kThreads), 0, s, mask, y, out, n, window, first);
    return hipGetLastError();
}

hipError_t launch_psnr(const float2* img, const float2* truth, long long npx, int n_images, double* terms,
                       hipStream_t s) {
    if (n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_psnr, dim3((unsigned)n_images), dim3(kPsnrThreads), 0, s, img, truth, npx, terms);
    return hipGetLastError();
}

}  // namespace vp
