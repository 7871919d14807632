// rhg_sample.hip -- point sampler (Algorithm 1, angular and radial draws);
// the draw itself is in rhg_sample.h.
#include "rhg_sample.h"

namespace rhg {

__global__ void __launch_bounds__(256) sample_kernel(int64_t n, uint32_t k0, uint32_t k1, double alpha,
                                                     double R, double c, double c_lo, double *__restrict__ r,
                                                     double *__restrict__ theta)
{
    __shared__ dd tab[LOGT_N];
    fill_log_table(tab, threadIdx.x, blockDim.x);
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double ri, ti;
        sample_point(i, k0, k1, alpha, R, c, c_lo, tab, &ri, &ti);
        theta[i] = ti;
        r[i] = ri;
    }
}
hipError_t launch_sample(const rhg_params &p, double *r, double *theta, hipStream_t s)
{
    if (p.n <= 0) return hipSuccess;
    // fewer, longer-running workgroups: each computes the log table once
    int64_t blocks = (p.n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p.n, (uint32_t)p.seed,
                       (uint32_t)(p.seed >> 32), p.alpha, p.R, p.cosh_aR_m1, p.cosh_aR_m1_lo, r, theta);
    return hipGetLastError();
}

}  // namespace rhg
