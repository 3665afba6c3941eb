// Issue-rate probe of the compute units (diagnostics): the measured basis of the
// roofline peaks the benchmark reports.  Every thread runs `iters` rounds of 16
// independent operations of one kind, so that with a few waves per SIMD a launch is
// bound by the rate at which the SIMDs (or the LDS) accept that kind.
#include "hsg_launch.h"

namespace hsg {
namespace {

constexpr int kProbeChains = 16;
constexpr int kProbeLds = 4096;  // floats of LDS per workgroup

template <int KIND>
__global__ void __launch_bounds__(1024) k_probe_issue(float* sink, int iters) {
    __shared__ float s[kProbeLds];
    for (int i = threadIdx.x; i < kProbeLds; i += blockDim.x) s[i] = static_cast<float>(i) * 1e-3f;
    __syncthreads();
    const float x = static_cast<float>(threadIdx.x) * 1e-7f, y = static_cast<float>(threadIdx.x) * 2e-7f;
    const double dx = x, dy = y;
    float a[kProbeChains];
    double d[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) {
        a[c] = static_cast<float>(c) * 1e-3f + x;
        d[c] = static_cast<double>(c) * 1e-3 + dx;
    }
    // LDS reads: wave w (mod 4) reads 64 consecutive words (kind 3) or 64 consecutive
    // 16-byte vectors (kind 4) per operation; largest index 3*64 + 63 + 256*15 = 4095
    // (kind 3) and 3*64 + 63 + 256*3 = 1023 vectors (kind 4), inside the array
    const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3;
    for (int it = 0; it < iters; ++it) {
        if constexpr (KIND == 0) {  // binary32 FMA
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) a[c] = fmaf(a[c], x, y);
        } else if constexpr (KIND == 1) {  // binary64 FMA
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) d[c] = fma(d[c], dx, dy);
        } else if constexpr (KIND == 2) {  // binary32 transcendental: 2^-a (a fixed point near 0.64)
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);
        } else if constexpr (KIND == 3) {  // LDS, 4-byte words
            asm volatile("" ::: "memory");  // the reads are made afresh each round
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) a[c] += s[w * 64 + lane + 256 * c];
        } else {  // LDS, 16-byte vectors
            asm volatile("" ::: "memory");
            const float4* s4 = reinterpret_cast<const float4*>(s);
#pragma unroll
            for (int c = 0; c < kProbeChains / 4; ++c) {
                const float4 v = s4[w * 64 + lane + 256 * c];
                a[4 * c] += v.x;
                a[4 * c + 1] += v.y;
                a[4 * c + 2] += v.z;
                a[4 * c + 3] += v.w;
            }
        }
    }
    float sum = 0.0f;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) sum += a[c] + static_cast<float>(d[c]);
    sink[static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x] = sum;
}

}  // namespace

hipError_t launch_probe_issue(int kind, int n_groups, int threads, int iters, float* sink, hipStream_t st) {
    const dim3 g(n_groups), b(threads);
    switch (kind) {
    case 0: hipLaunchKernelGGL(k_probe_issue<0>, g, b, 0, st, sink, iters); break;
    case 1: hipLaunchKernelGGL(k_probe_issue<1>, g, b, 0, st, sink, iters); break;
    case 2: hipLaunchKernelGGL(k_probe_issue<2>, g, b, 0, st, sink, iters); break;
    case 3: hipLaunchKernelGGL(k_probe_issue<3>, g, b, 0, st, sink, iters); break;
    default: hipLaunchKernelGGL(k_probe_issue<4>, g, b, 0, st, sink, iters); break;
    }
    return hipGetLastError();
}

}  // namespace hsg
