// The Newton pair shared by the all-pairs and batched kernels: one
// interaction of Eq. newton_force (the loop body of Sec. 3.3).
#pragma once

#include <hip/hip_runtime.h>

namespace pgh {

// 1/q from the transcendental unit (v_rcp_f32), which issues alongside the
// VALU; with GUARD a zero q gives 0 instead of inf.
template <bool GUARD>
__device__ __forceinline__ float rcp_of(float q)
{
    const float r = __builtin_amdgcn_rcpf(q);
    return GUARD ? ((q > 0.f) ? r : 0.f) : r;
}

template <bool REFINE, bool GUARD, bool PHI, bool RCP>
__device__ __forceinline__ void newton_pair(const float4 p, float px, float py, float pz,
                                            float pe, float &sx, float &sy, float &sz,
                                            float &sp)
{
    const float dx = p.x - px;
    const float dy = p.y - py;
    const float dz = p.z - pz;
    float q = __builtin_fmaf(dx, dx, pe);
    q = __builtin_fmaf(dy, dy, q);
    q = __builtin_fmaf(dz, dz, q);
    float y = __builtin_amdgcn_rsqf(q);
    if (GUARD) y = (q > 0.f) ? y : 0.f;
    float mr, mr3;
    if (REFINE) {
        const float y2 = y * y;
        const float t = __builtin_fmaf(q, y2, -3.0f);
        const float u = y * t;
        mr = p.w * u;  // p.w = -m/2
        if (RCP) {
            mr3 = mr * rcp_of<GUARD>(q);  // m rho / q
        } else {
            const float u2 = u * u;
            mr3 = mr * u2;  // 4 m rho^3
        }
    } else {
        mr = p.w * y;
        if (RCP) {
            mr3 = mr * rcp_of<GUARD>(q);
        } else {
            const float y2 = y * y;
            mr3 = mr * y2;
        }
    }
    if (PHI) sp -= mr;
    sx = __builtin_fmaf(mr3, dx, sx);
    sy = __builtin_fmaf(mr3, dy, sy);
    sz = __builtin_fmaf(mr3, dz, sz);
}

}  // namespace pgh
