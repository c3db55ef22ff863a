// Device helpers shared by the sweep kernels (rt_kernels.hip) and the plane-ordered
// sweep (rt_plane.hip): coordinate flips and ghost folding, and the first-order
// segment coefficients of section 3.3.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

namespace rtsc {
namespace {

// value of a per-axis quantity for a wave-uniform axis index
template <typename V>
__device__ __forceinline__ V sel3(int q, V x, V y, V z) { return q == 0 ? x : (q == 1 ? y : z); }

__device__ __forceinline__ int to_real(int g, int sg, int n) { return sg > 0 ? g : n - 1 - g; }

// One-step-outside index brought back in: wrap on periodic axes, clamp otherwise
// (selects, no branch).
__device__ __forceinline__ int fold(int x, int n, int periodic)
{
    const int lo = periodic ? x + n : 0, hi = periodic ? x - n : n - 1;
    return x < 0 ? lo : (x >= n ? hi : x);
}

// ---- segment integration -------------------------------------------------------
// FP64, plain form  I0 = I- E + psim S- + psi0 S0  with a source linear in tau:
// E = e^-dt, psi0 = 1 - (1 - e^-dt)/dt, psim = (1 - e^-dt) - psi0.  Below dt = 0.1
// psi0 comes from its Taylor series (Horner form) to avoid cancellation.
__device__ __forceinline__ void seg_coeffs(double dt, double &E, double &psim, double &psi0)
{
    const double e0 = -expm1(-dt);
    double p0;
    if (dt < 0.1) {
        // psi0 = dt/2! - dt^2/3! + dt^3/4! - ... (13 terms)
        const double c[13] = {1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0,
                              1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0,
                              1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
                              1.0 / 87178291200.0};
        double acc = c[12];
#pragma unroll
        for (int i = 11; i >= 0; --i) acc = c[i] - dt * acc;
        p0 = dt * acc;
    } else {
        p0 = 1.0 - e0 / dt;
    }
    E = exp(-dt);
    psi0 = p0;
    psim = e0 - p0;
}

// FP32, difference form  D0 = D- E + (S- - S0) g  with g = (1 - e^-dt)/dt = 1 - psi0,
// which is the plain form rewritten with D = I - S (E + psim + psi0 = 1).  One
// exponential, h = e^(-dt/2), gives both: E = h^2 and g = h sinh(y)/y with y = dt/2.
// Below dt = 0.5 the factor sinh(y)/y comes from its series 1 + y^2/3! + y^4/5! +
// y^6/7! in z = dt^2 (the next term is below 5e-11 there), which avoids the
// cancellation in 1 - E; above, g = (1 - E)/dt.
__device__ __forceinline__ void seg_coeffs(float dt, float &E, float &g)
{
    // both forms are evaluated and one is selected: no branch in the sweep step
    const float h = __builtin_amdgcn_exp2f(dt * -0.72134752f);   // 2^(-dt log2(e) / 2)
    E = h * h;
    const float z = dt * dt;
    float acc = fmaf(z, 1.0f / 322560.0f, 1.0f / 1920.0f);   // y^6/7!, y^4/5! in z
    acc = fmaf(z, acc, 1.0f / 24.0f);                          // y^2/3!
    const float gs = h * fmaf(z, acc, 1.0f);
    const float gc = (1.0f - E) * __builtin_amdgcn_rcpf(dt);
    g = dt < 0.5f ? gs : gc;
}

}  // namespace
}  // namespace rtsc
