// Small kernels around the force path: the self-term correction of raw
// potentials (Sec. 4.1).
#include <map>
#include <mutex>

#include "pgh_internal.h"

namespace pgh {

namespace {

// phi_i += m_i / eps_i: removes the self term -m_i/eps_i that the raw sum of
// an i-particle that is also a j-particle contains (Sec. 4.1).  A zero eps
// contributes nothing (the guarded kernel skips the zero-distance pair).
__global__ void __launch_bounds__(256) k_self_potential(int n, const float *__restrict__ m,
                                                        const float *__restrict__ eps2i,
                                                        float eps2_all, float *__restrict__ phi)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float e2 = eps2i ? eps2i[i] : eps2_all;
    if (e2 > 0.f) phi[i] += m[i] * __builtin_amdgcn_rsqf(e2);
}

}  // namespace

hipError_t launch_self_potential(int n, const float *m, const float *eps2i, float eps2_all,
                                 float *phi, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_self_potential, dim3((n + 255) / 256), dim3(256), 0, s, n, m, eps2i,
                       eps2_all, phi);
    return hipGetLastError();
}

hipError_t allow_dynamic_lds(const void *kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    static std::mutex mu;
    static std::map<const void *, size_t> allowed;
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = allowed[kernel];
    if (bytes <= have) return hipSuccess;
    const hipError_t e =
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) have = bytes;
    return e;
}

}  // namespace pgh
