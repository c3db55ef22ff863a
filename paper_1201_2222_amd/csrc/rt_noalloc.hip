// rt_formal_solve_noalloc: one formal solution J = Lambda[S] (section 3.3) with every
// internal buffer in a fixed-size device array of the library, for callers that
// cannot allocate device memory (code under graph capture, tight serving loops).
//
// It runs the kernels of rt_formal_solve on a freshly created problem: the tile
// wavefront of rt_kernels.hip over the same ray geometry, tile order and launch
// shape, with the periodic ghosts cold (S of the wrapped vertex).  Instead of
// per-problem allocations its state (ray table, tile list, FP32 chi, padded face
// planes, periodic memory, octant partial sums, per-bin control words) is carved
// out of `scratch`, a file-scope device array of kScratchBytes per GPU.  The ray
// geometry and the tile list are built on the device from kernel arguments, so the
// call needs no host buffer to outlive it either.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>

#include "../../include/rt.h"
#include "rt_internal.h"

namespace rtsc {

// from rt_api.cpp: the description checks of rt_problem_create, and the error text
// kept for rt_last_error
rt_status validate_desc(const rt_problem_desc *d, int *na_out);
void record_error(const char *msg);

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU
constexpr int kNoallocMaxRays = 80;                  // ray table passed as a kernel argument
constexpr int kMaxDevices = 64;

// the library-owned workspace; host code uses only the device addresses below
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each device

// Address of this device's copy of `scratch`, looked up once per device.
hipError_t scratch_address(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = ptr;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return hipSuccess;
}

// Rays in the caller's (or the generated) order, passed by value.
struct RayInput {
    double mu[kNoallocMaxRays][3];
    double w[kNoallocMaxRays];
    double h[3];
    int na;
};

// Per-ray short-characteristic geometry (section 3.3), octant-major and stable within
// an octant, written to rays[na]: the same arithmetic as the library's host-side
// construction (divisions and products only, nothing contracted), so the table is
// bitwise the one rt_problem_create builds.
__global__ void noalloc_geometry_kernel(RayInput in, RayGeo *rays)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int slot = 0;
    for (int o = 0; o < 8; ++o)
        for (int k = 0; k < in.na; ++k) {
            const double *m = in.mu[k];
            const int oct = (m[0] < 0.0 ? 1 : 0) | (m[1] < 0.0 ? 2 : 0) | (m[2] < 0.0 ? 4 : 0);
            if (oct != o) continue;
            double len[3];
            for (int q = 0; q < 3; ++q) len[q] = (m[q] == 0.0) ? __builtin_inf() : in.h[q] / fabs(m[q]);
            int d = 2;   // equal lengths: z before y before x
            if (len[1] < len[d]) d = 1;
            if (len[0] < len[d]) d = 0;
            RayGeo g{};
            g.d = d;
            g.a = (d == 0) ? 1 : 0;
            g.b = (d == 2) ? 1 : 2;
            g.oct = oct;
            g.gidx = k;
            g.s = len[d];
            const double fa = fmin(1.0, __dmul_rn(g.s, fabs(m[g.a])) / in.h[g.a]);
            const double fb = fmin(1.0, __dmul_rn(g.s, fabs(m[g.b])) / in.h[g.b]);
            g.w4[0] = __dmul_rn(1.0 - fa, 1.0 - fb);
            g.w4[1] = __dmul_rn(fa, 1.0 - fb);
            g.w4[2] = __dmul_rn(1.0 - fa, fb);
            g.w4[3] = __dmul_rn(fa, fb);
            g.fa = fa;
            g.fb = fb;
            g.wk = in.w[k];
            for (int q = 0; q < 3; ++q) g.mu[q] = m[q];
            rays[slot++] = g;
        }
}

// The tile list sorted by stage tx + ty + tz (within a stage: tz, then ty ascending),
// the order rt_problem_create uses; and zeroed per-bin control words.
__global__ void noalloc_tiles_kernel(int nt0, int nt1, int nt2, int *tiles, int *ctl, int nctl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int k = 0;
        for (int s = 0; s < nt0 + nt1 + nt2 - 2; ++s)
            for (int tz = 0; tz < nt2; ++tz)
                for (int ty = 0; ty < nt1; ++ty) {
                    const int tx = s - ty - tz;
                    if (tx >= 0 && tx < nt0) tiles[k++] = tx | (ty << 10) | (tz << 20);
                }
    }
    for (int i = threadIdx.x; i < nctl; i += blockDim.x) ctl[i] = 0;
}

thread_local char g_noalloc_err[512];

rt_status nfail(rt_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_noalloc_err, sizeof g_noalloc_err, fmt, ap);
    va_end(ap);
    rtsc::record_error(g_noalloc_err);
    return s;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

template <typename Real>
rt_status noalloc_run(const rt_problem_desc *d, int na, const RayInput &rin, const double *chi, const double *B,
                      const double *S, double *J, double *lambda_star, unsigned char *base, hipStream_t st)
{
    const bool f32 = sizeof(Real) == 4;
    SweepArgs<Real> A{};
    const int n[3] = {d->nx, d->ny, d->nz};
    int nt[3];
    for (int q = 0; q < 3; ++q) nt[q] = (n[q] + kTile - 1) / kTile;
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const int64_t nc = cells * d->nf;
    const int ntiles = nt[0] * nt[1] * nt[2];
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += align256(bytes);
        return p;
    };
    RayGeo *rays = reinterpret_cast<RayGeo *>(carve(sizeof(RayGeo) * na));
    int *tiles = reinterpret_cast<int *>(carve(sizeof(int) * ntiles));
    int *ctl = reinterpret_cast<int *>(carve(sizeof(int) * 2 * d->nf));   // frozen, parity
    const Real *chiR = nullptr;
    if (f32) {
        float *c32 = reinterpret_cast<float *>(carve(sizeof(float) * nc));
        if (launch_convert_f32(chi, c32, nc, st) != hipSuccess) return nfail(RT_E_HIP, "chi conversion launch failed");
        chiR = reinterpret_cast<const Real *>(c32);
    } else {
        chiR = reinterpret_cast<const Real *>(chi);
    }
    for (int q = 0; q < 3; ++q) {
        A.n[q] = n[q];
        A.nt[q] = nt[q];
        A.bc_lo[q] = d->bc_lo[q];
        A.bc_hi[q] = d->bc_hi[q];
        A.periodic[q] = d->bc_lo[q] == RT_BC_PERIODIC;
    }
    A.plane[0] = (int64_t)n[1] * n[2];
    A.plane[1] = (int64_t)n[0] * n[2];
    A.plane[2] = (int64_t)n[0] * n[1];
    A.pplane[0] = FacePlane(n[1], n[2]).slot();
    A.pplane[1] = FacePlane(n[0], n[2]).slot();
    A.pplane[2] = FacePlane(n[0], n[1]).slot();
    for (int q = 0; q < 3; ++q) {
        A.face[q] = reinterpret_cast<Real *>(carve(sizeof(Real) * (size_t)d->nf * na * nt[q] * A.pplane[q]));
        A.wrap[q] = A.periodic[q] ? reinterpret_cast<double *>(carve(sizeof(double) * (size_t)d->nf * na * 2 * A.plane[q]))
                                  : nullptr;
    }
    Real *part = reinterpret_cast<Real *>(carve(sizeof(Real) * 8 * (size_t)nc));
    A.nf = d->nf;
    A.na = na;
    A.R = na / 8;
    A.cells = cells;
    A.rays = rays;
    A.chi = chiR;
    A.S = S;
    A.B = B;
    for (int k = 0; k < 6; ++k) A.fixed[k] = d->I_fixed[k];
    A.part = part;
    A.f0 = 0;
    A.nfc = d->nf;
    A.tiles = tiles;
    A.frozen = ctl;
    A.parity = ctl + d->nf;
    A.stage_tab = nullptr;
    A.nstages = nt[0] + nt[1] + nt[2] - 2;
    A.order = d->order;
    A.noct = 8;

    hipLaunchKernelGGL(noalloc_geometry_kernel, dim3(1), dim3(64), 0, st, rin, rays);
    hipLaunchKernelGGL(noalloc_tiles_kernel, dim3(1), dim3(256), 0, st, nt[0], nt[1], nt[2], tiles, ctl, 2 * d->nf);
    if (hipGetLastError() != hipSuccess) return nfail(RT_E_HIP, "set-up launch failed");
    if (launch_periodic_cold<Real>(A, st) != hipSuccess) return nfail(RT_E_HIP, "periodic set-up launch failed");
    if (launch_ghost_fill<Real>(A, st) != hipSuccess) return nfail(RT_E_HIP, "ghost launch failed");

    // launch shape of rt_problem_create: one wave per ray of an octant, at most
    // kMaxWaves, fewer if the LDS of the device does not hold them
    int dev = 0, lds_limit = 65536;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipGetLastError();
    int waves = std::min(A.R, kMaxWaves);
    while (waves > 1 && sweep_lds_bytes((int)sizeof(Real), waves, 1, A.R > waves, d->order) > (size_t)lds_limit) --waves;
    if (sweep_lds_bytes((int)sizeof(Real), waves, 1, A.R > waves, d->order) > (size_t)lds_limit)
        return nfail(RT_E_UNSUPPORTED, "the sweep needs more LDS than the device allows");

    // stage offsets of the tile list (the same arithmetic as the device's list)
    int stage_off = 0;
    for (int s = 0; s < A.nstages; ++s) {
        int cnt = 0;
        for (int tz = 0; tz < nt[2]; ++tz)
            for (int ty = 0; ty < nt[1]; ++ty) {
                const int tx = s - ty - tz;
                if (tx >= 0 && tx < nt[0]) ++cnt;
            }
        A.stage_off = stage_off;
        A.stage_cnt = cnt;
        A.stage = s;
        hipError_t e;
        if constexpr (sizeof(Real) == 4)
            e = launch_sweep_stage_f32(A, waves, 1, st);
        else
            e = launch_sweep_stage_f64(A, waves, 1, st);
        if (e != hipSuccess) return nfail(RT_E_HIP, "sweep launch failed: %s", hipGetErrorString(e));
        stage_off += cnt;
    }
    if (launch_partial_sum<Real>(part, 8, S, f32 ? 1 : 0, d->nf, cells, nullptr, J, st) != hipSuccess)
        return nfail(RT_E_HIP, "partial-sum launch failed");
    if (lambda_star &&
        launch_lambda_star(n, d->bc_lo, d->bc_hi, d->nf, na, d->order, rays, chi, lambda_star, st) != hipSuccess)
        return nfail(RT_E_HIP, "Lambda* launch failed");
    return RT_OK;
}

}  // namespace

// Scratch bytes the no-allocation formal solution needs for this description (the
// carving of noalloc_run).
size_t noalloc_bytes(const rt_problem_desc *d, int na)
{
    const int n[3] = {d->nx, d->ny, d->nz};
    int nt[3];
    for (int q = 0; q < 3; ++q) nt[q] = (n[q] + kTile - 1) / kTile;
    const size_t cells = (size_t)n[0] * n[1] * n[2], nc = cells * d->nf;
    const size_t rs = d->precision == RT_F32 ? 4 : 8;
    const size_t plane[3] = {(size_t)n[1] * n[2], (size_t)n[0] * n[2], (size_t)n[0] * n[1]};
    const size_t pplane[3] = {(size_t)FacePlane(n[1], n[2]).slot(), (size_t)FacePlane(n[0], n[2]).slot(),
                              (size_t)FacePlane(n[0], n[1]).slot()};
    size_t b = align256(sizeof(RayGeo) * na) + align256(sizeof(int) * nt[0] * nt[1] * nt[2]) +
               align256(sizeof(int) * 2 * d->nf);
    if (rs == 4) b += align256(4 * nc);
    for (int q = 0; q < 3; ++q) {
        b += align256(rs * (size_t)d->nf * na * nt[q] * pplane[q]);
        if (d->bc_lo[q] == RT_BC_PERIODIC) b += align256(8 * (size_t)d->nf * na * 2 * plane[q]);
    }
    b += align256(rs * 8 * nc);
    return b;
}

size_t noalloc_capacity() { return kScratchBytes; }

}  // namespace rtsc

using namespace rtsc;

extern "C" rt_status rt_formal_solve_noalloc(const rt_problem_desc *desc, const void *chi, const void *B,
                                             const void *S, void *J, void *lambda_star, void *stream)
{
    int na = 0;
    rt_status s = validate_desc(desc, &na);
    if (s != RT_OK) return s;
    if (desc->schedule == RT_SCHED_PERSISTENT)
        return nfail(RT_E_UNSUPPORTED, "the no-allocation call runs the staged schedule (one launch per hyperplane)");
    if (!chi || !B || !S || !J) return nfail(RT_E_INVALID, "chi, B, S and J are required");
    if (desc->in_dtype != RT_DTYPE_F64) return nfail(RT_E_UNSUPPORTED, "the no-allocation call takes FP64 arrays");
    if (desc->interp != RT_INTERP_BILINEAR)
        return nfail(RT_E_UNSUPPORTED, "the no-allocation call runs the tile wavefront (bilinear upwind intensity)");
    if (na > kNoallocMaxRays) return nfail(RT_E_UNSUPPORTED, "the no-allocation call takes at most %d rays", kNoallocMaxRays);
    const size_t need = noalloc_bytes(desc, na);
    if (need > kScratchBytes)
        return nfail(RT_E_UNSUPPORTED, "the problem needs %zu bytes of workspace, the no-allocation call has %zu", need,
                     kScratchBytes);
    RayInput rin{};
    rin.na = na;
    rin.h[0] = desc->dx;
    rin.h[1] = desc->dy;
    rin.h[2] = desc->dz;
    if (desc->mu) {
        for (int k = 0; k < na; ++k) {
            for (int q = 0; q < 3; ++q) rin.mu[k][q] = desc->mu[3 * k + q];
            rin.w[k] = desc->w[k];
        }
    } else {
        s = rt_quadrature(desc->n_mu, &rin.mu[0][0], rin.w, &na);
        if (s != RT_OK) return s;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return nfail(RT_E_HIP, "no current HIP device");
    }
    unsigned char *base = nullptr;
    const hipError_t e = scratch_address(dev, &base);
    if (e != hipSuccess) return nfail(RT_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double *chi64 = static_cast<const double *>(chi);
    if (desc->precision == RT_F32)
        return noalloc_run<float>(desc, na, rin, chi64, static_cast<const double *>(B), static_cast<const double *>(S),
                                  static_cast<double *>(J), static_cast<double *>(lambda_star), base, st);
    return noalloc_run<double>(desc, na, rin, chi64, static_cast<const double *>(B), static_cast<const double *>(S),
                               static_cast<double *>(J), static_cast<double *>(lambda_star), base, st);
}
