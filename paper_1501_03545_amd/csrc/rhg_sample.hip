// rhg_sample.hip -- point sampler (Algorithm 1, angular and radial draws).
//
// Vertex i draws its two uniforms from Philox4x32-10 (Salmon, Moraes, Dror,
// Shaw, SC'11) with counter (i_lo, i_hi, 0, 0) and key (seed_lo, seed_hi):
// one 128-bit block gives two 53-bit uniforms.  The angle is uniform on
// [0, 2 pi) and the radius follows Eq. (1) by inverting its CDF
// F(r) = (cosh(alpha r) - 1) / (cosh(alpha R) - 1) (Appendix C with the full
// angular range): r = acosh(1 + u (cosh(alpha R) - 1)) / alpha, evaluated as
// log1p(x + sqrt(x (x + 2))) / alpha with x = u (cosh(alpha R) - 1), which
// keeps full relative accuracy for small u.  The radius is evaluated in
// double-double (about 104 bits) and rounded once, so it is the correctly
// rounded binary64 value unless the exact radius lies within about 2^-100
// (relative) of a rounding boundary.
#include "rhg_internal.h"
#include "rhg_philox.h"

namespace rhg {

__global__ void __launch_bounds__(256) sample_kernel(int64_t n, uint32_t k0, uint32_t k1, double alpha,
                                                     double R, double c, double c_lo, double *__restrict__ r,
                                                     double *__restrict__ theta)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t x0 = (uint32_t)(uint64_t)i, x1 = (uint32_t)((uint64_t)i >> 32), x2 = 0u, x3 = 0u;
        philox4x32_10(x0, x1, x2, x3, k0, k1);
        const uint64_t a = ((uint64_t)x1 << 32) | x0;
        const uint64_t b = ((uint64_t)x3 << 32) | x2;
        const double ut = (double)(a >> 11) * 0x1p-53;
        const double ur = (double)(b >> 11) * 0x1p-53;
        theta[i] = RHG_TWO_PI_D * ut;
        const dd x = dd_mul_d(dd_make(c, c_lo), ur);
        const dd y = dd_add(x, dd_sqrt(dd_mul(x, dd_add_d(x, 2.0))));
        const dd ri = dd_div_d(dd_log1p(y), alpha);
        r[i] = fmin(ri.hi, R);  // the exact value is <= R
    }
}

hipError_t launch_sample(const rhg_params &p, double *r, double *theta, hipStream_t s)
{
    if (p.n <= 0) return hipSuccess;
    int64_t blocks = (p.n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(sample_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p.n, (uint32_t)p.seed,
                       (uint32_t)(p.seed >> 32), p.alpha, p.R, p.cosh_aR_m1, p.cosh_aR_m1_lo, r, theta);
    return hipGetLastError();
}

}  // namespace rhg
