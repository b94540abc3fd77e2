// Test pin: accuracy of the gfx950 hardware transcendentals the FP32 Box-Muller
// transform and accept test use, over every 24-bit uniform u = (f + 1) 2^-24:
// v_cos_f32 / v_sin_f32 (argument in revolutions) against cos/sin(2 pi u) in
// FP64, v_log_f32 (log2) scaled to ln, and v_sqrt_f32.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
__device__ unsigned int g_err[4];   // bit patterns of the non-negative float maxima: |cos err|, |sin err|, rel ln err, rel sqrt err
__global__ void probe(unsigned int n)
{
    const unsigned int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    const float u = static_cast<float>(f + 1u) * 5.9604644775390625e-08f;
    double sd, cd;
    sincospi(2.0 * static_cast<double>(u), &sd, &cd);
    const float c = __builtin_amdgcn_cosf(u), s = __builtin_amdgcn_sinf(u);
    const float l = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
    const double ld = log(static_cast<double>(u));
    const float e_c = static_cast<float>(fabs(static_cast<double>(c) - cd));
    const float e_s = static_cast<float>(fabs(static_cast<double>(s) - sd));
    const float e_l = (ld != 0.0) ? static_cast<float>(fabs((static_cast<double>(l) - ld) / ld)) : static_cast<float>(fabs(l));
    const float x = -2.0f * l;
    const float r = __builtin_amdgcn_sqrtf(x);
    const double rd = sqrt(static_cast<double>(x));
    const float e_r = (rd != 0.0) ? static_cast<float>(fabs((static_cast<double>(r) - rd) / rd)) : 0.0f;
    atomicMax(&g_err[0], __float_as_uint(e_c));
    atomicMax(&g_err[1], __float_as_uint(e_s));
    atomicMax(&g_err[2], __float_as_uint(e_l));
    atomicMax(&g_err[3], __float_as_uint(e_r));
}
int main()
{
    const unsigned int n = 1u << 24;
    unsigned int z[4] = {0, 0, 0, 0};
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_err), z, sizeof(z)) != hipSuccess) return 1;
    hipLaunchKernelGGL(probe, dim3(n / 256), dim3(256), 0, 0, n);
    if (hipDeviceSynchronize() != hipSuccess) return 2;
    unsigned int e[4];
    if (hipMemcpyFromSymbol(e, HIP_SYMBOL(g_err), sizeof(e)) != hipSuccess) return 3;
    float v[4];
    for (int i = 0; i < 4; ++i) { unsigned int b = e[i]; __builtin_memcpy(&v[i], &b, 4); }
    std::printf("max |cos err| %.3e  max |sin err| %.3e  max rel ln err %.3e  max rel sqrt err %.3e\n", v[0], v[1], v[2], v[3]);
    return 0;
}
