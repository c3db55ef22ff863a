// HIP kernels of the short-characteristics formal solution (section 3.3), the
// diagonal Lambda* and the Jacobi ALI update (section 3.4) for gfx950.
//
// Sweep organisation.  Per octant every ray depends only on upwind vertices, so
// in the octant's "flipped" coordinates (each axis reversed where the octant's
// direction is negative) all dependencies point to lower coordinates.  The grid is
// cut into T^3 tiles; a tile depends on its upwind neighbour tiles, so tiles with
// the same tx + ty + tz (one "stage") are independent and run in one launch.
// Inside a tile each wave takes one ray at a time and sweeps plane by plane along
// the axis that ray crosses first: all upwind vertices of a plane lie in the
// previous plane, so the 64 lanes of the wave update a whole T x T plane at once.
// chi and S of the tile plus its upwind halo are staged in LDS once and shared by
// all rays of the octant; the previous plane of I lives in a small per-wave LDS
// buffer; neighbour tiles exchange their downwind faces through global memory.
#include <hip/hip_runtime.h>

#include "rt_internal.h"

namespace rtsc {

namespace {

constexpr int T = kTile;
constexpr int TP = T + 1;            // tile plus one upwind halo layer
constexpr int TILE_LDS = TP * TP * TP;
constexpr int PLANE_LDS = TP * TP;

__device__ __forceinline__ void wave_lds_sync()
{
    // make this wave's LDS stores visible to its other lanes (lgkmcnt(0)) and keep
    // the compiler from moving LDS accesses across this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int64_t plane_index(int q, const int v[3], const int n[3])
{
    // plane normal to axis q: the other two axes in increasing order, lower one fastest
    const int p1 = (q == 0) ? 1 : 0;
    const int p2 = (q == 2) ? 1 : 2;
    return (int64_t)v[p2] * n[p1] + v[p1];
}

__device__ __forceinline__ int to_real(int g, int sg, int n) { return sg > 0 ? g : n - 1 - g; }

// One-step-outside index brought back in: wrap on periodic axes, clamp otherwise.
__device__ __forceinline__ int fold(int x, int n, int periodic)
{
    if (x >= 0 && x < n) return x;
    if (periodic) return x < 0 ? x + n : x - n;
    return x < 0 ? 0 : n - 1;
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
        double acc;
        const double c[13] = {1.0 / 2.0, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0,
                              1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0,
                              1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0,
                              1.0 / 87178291200.0};
        acc = c[12];
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
// which is the plain form rewritten with D = I - S (E + psim + psi0 = 1).  g comes
// from its Taylor series sum_n (-dt)^n/(n+1)! below dt = 0.5 (9 terms).
__device__ __forceinline__ void seg_coeffs(float dt, float &E, float &g)
{
    E = __expf(-dt);
    if (dt < 0.5f) {
        float acc = 1.0f / 3628800.0f;                    // 1/10!
        acc = 1.0f / 362880.0f - dt * acc;                // 1/9!
        acc = 1.0f / 40320.0f - dt * acc;
        acc = 1.0f / 5040.0f - dt * acc;
        acc = 1.0f / 720.0f - dt * acc;
        acc = 1.0f / 120.0f - dt * acc;
        acc = 1.0f / 24.0f - dt * acc;
        acc = 1.0f / 6.0f - dt * acc;
        acc = 0.5f - dt * acc;
        g = 1.0f - dt * acc;
    } else {
        g = (1.0f - E) * __builtin_amdgcn_rcpf(dt);
    }
}

template <typename Real, bool DFORM>
struct Tile {
    const SweepArgs<Real> &A;
    int oct, f, par;
    int sg[3], t[3], g0[3], ext[3];
    const Real *SL;
    int64_t fbase;  // f * cells

    __device__ Tile(const SweepArgs<Real> &A_) : A(A_) {}

    __device__ __forceinline__ int lds_index(const int gv[3]) const
    {
        return ((gv[2] - g0[2] + 1) * TP + (gv[1] - g0[1] + 1)) * TP + (gv[0] - g0[0] + 1);
    }

    __device__ __forceinline__ int64_t face_offset(int q, int ray, int slot) const
    {
        return (((int64_t)f * A.na + ray) * (A.nt[q] + 1) + slot) * A.plane[q];
    }

    // Value (I, or D = I - S) at a halo vertex gv (flipped coordinates) just upwind
    // of this tile, for the given ray.
    __device__ Real halo(const int gv[3], int ray, int gidx) const
    {
        bool out[3];
        bool any = false;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            out[q] = gv[q] < 0;
            any |= out[q];
        }
        if (!any) {
            // a vertex of an upwind neighbour tile: read that tile's downwind face
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (gv[q] == g0[q] - 1)
                    return A.face[q][face_offset(q, ray, t[q] - 1) + plane_index(q, gv, A.n)];
            return Real(0);
        }
        const Real Sg = SL[lds_index(gv)];
        // a ghost outside a non-periodic face: that face's boundary condition,
        // the highest axis first
#pragma unroll
        for (int q = 2; q >= 0; --q) {
            if (!out[q] || A.periodic[q]) continue;
            const int kind = (sg[q] > 0) ? A.bc_lo[q] : A.bc_hi[q];
            double I = 0.0;
            if (kind == BC_THERMAL || kind == BC_FIXED) {
                int u[3];
#pragma unroll
                for (int p = 0; p < 3; ++p)
                    u[p] = fold(to_real(gv[p], sg[p], A.n[p]), A.n[p], A.periodic[p]);
                if (kind == BC_THERMAL) {
                    I = A.B[fbase + ((int64_t)u[2] * A.n[1] + u[1]) * A.n[0] + u[0]];
                } else {
                    const double *F = A.fixed[2 * q + (sg[q] > 0 ? 0 : 1)];
                    I = F[((int64_t)f * A.na + gidx) * A.plane[q] + plane_index(q, u, A.n)];
                }
            }
            return DFORM ? Real(I) - Sg : Real(I);
        }
        // only periodic axes are outside: the previous sweep's intensity at the
        // wrapped vertex, kept on the ray's outgoing plane
        int w[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) w[q] = out[q] ? A.n[q] - 1 : gv[q];
        int q = out[0] ? 0 : (out[1] ? 1 : 2);
        const Real I = A.face[q][face_offset(q, ray, A.nt[q] - 1 + par) + plane_index(q, w, A.n)];
        return DFORM ? I - Sg : I;
    }
};

// dynamic LDS of one sweep workgroup with W waves: chi and S tiles, two plane
// buffers per wave, one partial-sum tile per wave
template <typename Real>
constexpr size_t sweep_lds_bytes(int W)
{
    return sizeof(Real) * (2 * (size_t)TILE_LDS + (size_t)W * (2 * PLANE_LDS + T * T * T));
}

template <typename Real, bool DFORM>
__global__ void __launch_bounds__(64 * kMaxWaves) sweep_stage_kernel(SweepArgs<Real> A)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Real *chiL = reinterpret_cast<Real *>(lds_raw);
    Real *SLs = chiL + TILE_LDS;
    Real *PlBase = SLs + TILE_LDS;
    const int Wn = blockDim.x >> 6;
    Real *JwBase = PlBase + (size_t)Wn * 2 * PLANE_LDS;

    const int oct = blockIdx.x & 7;
    const int item = blockIdx.x >> 3;
    const int f = blockIdx.y;
    if (A.frozen[f]) return;

    Tile<Real, DFORM> tl(A);
    tl.oct = oct;
    tl.f = f;
    tl.par = A.parity[f];
    tl.fbase = (int64_t)f * A.cells;
    tl.SL = SLs;
    const int packed = A.tiles[A.stage_off + item];
    tl.t[0] = packed & 1023;
    tl.t[1] = (packed >> 10) & 1023;
    tl.t[2] = (packed >> 20) & 1023;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        tl.sg[q] = (oct >> q) & 1 ? -1 : 1;
        tl.g0[q] = tl.t[q] * T;
        tl.ext[q] = min(T, A.n[q] - tl.g0[q]);
    }

    // ---- stage chi and S of the tile and its upwind halo in LDS --------------------
    const Real *chif = A.chi + tl.fbase;
    const Real *Sf = A.S + tl.fbase;
    for (int idx = threadIdx.x; idx < TILE_LDS; idx += blockDim.x) {
        const int l[3] = {idx % TP, (idx / TP) % TP, idx / (TP * TP)};
        int u[3];
        bool skip = false;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int g = tl.g0[q] + l[q] - 1;
            skip |= (l[q] > tl.ext[q]);
            u[q] = fold(to_real(g, tl.sg[q], A.n[q]), A.n[q], A.periodic[q]);
        }
        if (skip) continue;
        const int64_t c = ((int64_t)u[2] * A.n[1] + u[1]) * A.n[0] + u[0];
        chiL[idx] = chif[c];
        SLs[idx] = Sf[c];
    }
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int W = Wn;
    Real *Jmine = JwBase + (size_t)wave * T * T * T;
    for (int c = lane; c < T * T * T; c += 64) Jmine[c] = Real(0);
    __syncthreads();

    // ---- per-wave ray sweeps ---------------------------------------------------------
    for (int r = wave; r < A.R; r += W) {
        const int ray = oct * A.R + r;
        const RayGeo &G = A.rays[ray];
        const int d = G.d, a = G.a, b = G.b;
        const Real s_half = Real(0.5 * G.s);
        const Real w00 = Real(G.w4[0]), w10 = Real(G.w4[1]), w01 = Real(G.w4[2]), w11 = Real(G.w4[3]);
        const Real wk = Real(G.wk);
        const int ed = tl.ext[d], ea = tl.ext[a], eb = tl.ext[b];
        // LDS strides of the d, a, b axes inside the staged tile
        const int str[3] = {1, TP, TP * TP};
        const int sd = str[d], sa = str[a], sb = str[b];
        Real *P0 = PlBase + (size_t)wave * 2 * PLANE_LDS;
        Real *P1 = P0 + PLANE_LDS;

        // upwind d-face of the tile (d = -1), with its a and b halo lines
        for (int e = lane; e < (ea + 1) * (eb + 1); e += 64) {
            const int ia = e % (ea + 1) - 1, ib = e / (ea + 1) - 1;
            int gv[3];
            gv[d] = tl.g0[d] - 1;
            gv[a] = tl.g0[a] + ia;
            gv[b] = tl.g0[b] + ib;
            P0[(ia + 1) + (ib + 1) * TP] = tl.halo(gv, ray, G.gidx);
        }
        wave_lds_sync();

        for (int p = 0; p < ed; ++p) {
            const Real *Pp = (p & 1) ? P1 : P0;
            Real *Pc = (p & 1) ? P0 : P1;
            for (int c = lane; c < ea * eb; c += 64) {
                const int ia = c % ea, ib = c / ea;
                // staged-tile index of this vertex and of its upwind face vertices
                const int l0 = (p + 1) * sd + (ia + 1) * sa + (ib + 1) * sb;
                const int lu = l0 - sd;
                const int i00 = lu, i10 = lu - sa, i01 = lu - sb, i11 = lu - sa - sb;
                const int q00 = (ia + 1) + (ib + 1) * TP;
                const Real Im = w00 * Pp[q00] + w10 * Pp[q00 - 1] + w01 * Pp[q00 - TP] + w11 * Pp[q00 - TP - 1];
                const Real Sm = w00 * SLs[i00] + w10 * SLs[i10] + w01 * SLs[i01] + w11 * SLs[i11];
                const Real Cm = w00 * chiL[i00] + w10 * chiL[i10] + w01 * chiL[i01] + w11 * chiL[i11];
                const Real S0 = SLs[l0];
                const Real dt = s_half * (Cm + chiL[l0]);
                Real v;
                if constexpr (DFORM) {
                    Real E, g;
                    seg_coeffs(dt, E, g);
                    v = Im * E + (Sm - S0) * g;
                } else {
                    Real E, pm, p0;
                    seg_coeffs(dt, E, pm, p0);
                    v = Im * E + pm * Sm + p0 * S0;
                }
                Pc[q00] = v;
                int lc[3];
                lc[d] = p;
                lc[a] = ia;
                lc[b] = ib;
                Jmine[(lc[2] * T + lc[1]) * T + lc[0]] += wk * v;

                // downwind faces for the neighbour tiles / the next sweep's periodic ghosts
                const bool on_a = (ia == ea - 1), on_b = (ib == eb - 1), on_d = (p == ed - 1);
                if (on_a || on_b || on_d) {
                    int gv[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) gv[q] = tl.g0[q] + lc[q];
                    const int qs[3] = {a, b, d};
                    const bool on[3] = {on_a, on_b, on_d};
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        if (!on[k]) continue;
                        const int q = qs[k];
                        int slot;
                        Real val = v;
                        if (tl.t[q] < A.nt[q] - 1) {
                            slot = tl.t[q];
                        } else if (A.periodic[q]) {
                            slot = A.nt[q] - 1 + (tl.par ^ 1);
                            if constexpr (DFORM) val = v + S0;  // periodic memory keeps I
                        } else {
                            continue;
                        }
                        A.face[q][tl.face_offset(q, ray, slot) + plane_index(q, gv, A.n)] = val;
                    }
                }
            }
            // halo lines of plane p for the next step
            if (p + 1 < ed) {
                for (int e = lane; e < ea + eb + 1; e += 64) {
                    int ia, ib;
                    if (e <= eb) {
                        ia = -1;
                        ib = e - 1;
                    } else {
                        ia = e - eb - 1;
                        ib = -1;
                    }
                    int gv[3];
                    gv[d] = tl.g0[d] + p;
                    gv[a] = tl.g0[a] + ia;
                    gv[b] = tl.g0[b] + ib;
                    Pc[(ia + 1) + (ib + 1) * TP] = tl.halo(gv, ray, G.gidx);
                }
            }
            wave_lds_sync();
        }
    }
    __syncthreads();

    // ---- fixed-order sum over the waves -> this octant's partial sums --------------
    Real *outp = A.part + ((int64_t)oct * A.nf + f) * A.cells;
    for (int c = threadIdx.x; c < T * T * T; c += blockDim.x) {
        const int lc[3] = {c % T, (c / T) % T, c / (T * T)};
        if (lc[0] >= tl.ext[0] || lc[1] >= tl.ext[1] || lc[2] >= tl.ext[2]) continue;
        Real acc = JwBase[c];
        for (int w = 1; w < W; ++w) acc += JwBase[(size_t)w * T * T * T + c];
        int u[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) u[q] = to_real(tl.g0[q] + lc[q], tl.sg[q], A.n[q]);
        outp[((int64_t)u[2] * A.n[1] + u[1]) * A.n[0] + u[0]] = acc;
    }
}

// ---- Lambda*: diagonal of the formal-solution operator (section 3.4) -----------------
// Lambda*_ii = sum_k w_k psi0_k: the weight of S at the vertex itself in its own
// update.  psi0 depends only on the upwind chi, so this is a pointwise kernel.
__global__ void lambda_star_kernel(int nx, int ny, int nz, int bx0, int bx1, int by0, int by1, int bz0,
                                   int bz1, int nf, int na, const RayGeo *rays, const double *chi,
                                   double *lam)
{
    const int64_t cells = (int64_t)nx * ny * nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * nf) return;
    const int f = (int)(i / cells);
    const int64_t c = i - (int64_t)f * cells;
    const int n[3] = {nx, ny, nz};
    const int per[3] = {bx0 == BC_PERIODIC, by0 == BC_PERIODIC, bz0 == BC_PERIODIC};
    (void)bx1; (void)by1; (void)bz1;
    const int x[3] = {(int)(c % nx), (int)((c / nx) % ny), (int)(c / ((int64_t)nx * ny))};
    const double *cf = chi + (int64_t)f * cells;
    const double c0 = cf[c];
    double acc = 0.0;
    for (int k = 0; k < na; ++k) {
        const RayGeo &G = rays[k];
        int sg[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) sg[q] = (G.oct >> q) & 1 ? -1 : 1;
        double cm = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int u[3] = {x[0], x[1], x[2]};
            u[G.d] -= sg[G.d];
            u[G.a] -= (v & 1) * sg[G.a];
            u[G.b] -= (v >> 1) * sg[G.b];
#pragma unroll
            for (int q = 0; q < 3; ++q) u[q] = fold(u[q], n[q], per[q]);
            cm += G.w4[v] * cf[((int64_t)u[2] * ny + u[1]) * nx + u[0]];
        }
        double E, pm, p0;
        seg_coeffs(0.5 * G.s * (cm + c0), E, pm, p0);
        acc += G.wk * p0;
    }
    lam[i] = acc;
}

template <typename Real>
__global__ void periodic_cold_kernel(SweepArgs<Real> A, int q)
{
    // slot about to be read: nt_q - 1 + parity[f]; value S of the wrapped vertex
    const int64_t P = A.plane[q];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ray = blockIdx.y;
    const int f = blockIdx.z;
    if (i >= P) return;
    const int oct = A.rays[ray].oct;
    const int p1 = (q == 0) ? 1 : 0;
    const int p2 = (q == 2) ? 1 : 2;
    int gv[3];
    gv[q] = A.n[q] - 1;
    gv[p1] = (int)(i % A.n[p1]);
    gv[p2] = (int)(i / A.n[p1]);
    int u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = to_real(gv[k], (oct >> k) & 1 ? -1 : 1, A.n[k]);
    const Real Sv = A.S[(int64_t)f * A.cells + ((int64_t)u[2] * A.n[1] + u[1]) * A.n[0] + u[0]];
    const int slot = A.nt[q] - 1 + A.parity[f];
    A.face[q][(((int64_t)f * A.na + ray) * (A.nt[q] + 1) + slot) * P + i] = Sv;
}

template <typename Real>
__global__ void partial_sum_kernel(const Real *part, const double *S, int dform, int nf, int64_t cells,
                                   const int *frozen, double *J)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * nf) return;
    const int f = (int)(i / cells);
    if (frozen && frozen[f]) return;
    const int64_t stride = (int64_t)nf * cells;
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < 8; ++o) acc += (double)part[o * stride + i];
    J[i] = dform ? S[i] + acc : acc;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Jacobi update (eq. dsjacobi) and the per-bin residual max |dS|/S^{n+1} (eq. conv),
// both in FP64.  With dform the partials hold sum w (I - S), so J - S is summed
// without cancellation.
template <typename Real>
__global__ void __launch_bounds__(256) ali_update_kernel(const Real *part, int dform, int nf, int64_t cells,
                                                         const double *B, const double *eps,
                                                         const double *lam, double *S64, float *S32,
                                                         double *Jout, AliCtl ctl)
{
    __shared__ unsigned long long red[4];
    const int f = blockIdx.y;
    if (ctl.frozen[f]) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long rb = 0ull;
    if (c < cells) {
        const int64_t i = (int64_t)f * cells + c;
        const int64_t stride = (int64_t)nf * cells;
        double sum = 0.0;
#pragma unroll
        for (int o = 0; o < 8; ++o) sum += (double)part[o * stride + i];
        const double S = S64[i], e = eps[i];
        double num;
        if (dform) {
            num = (1.0 - e) * sum + e * (B[i] - S);
            Jout[i] = S + sum;
        } else {
            num = (1.0 - e) * sum + e * B[i] - S;
            Jout[i] = sum;
        }
        const double dS = num / (1.0 - (1.0 - e) * lam[i]);
        const double Sn = S + dS;
        S64[i] = Sn;
        if (S32) S32[i] = (float)Sn;
        const double r = (Sn != 0.0) ? fabs(dS) / fabs(Sn) : 0.0;
        rb = (unsigned long long)__double_as_longlong(r);
    }
    rb = wave_max_u64(rb);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rb;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] > m ? red[w] : m;
        if (m) atomicMax(&ctl.res_bits[f], m);
    }
}

__global__ void ali_finalize_kernel(AliCtl ctl, int nf, double delta_c, int per_bin_stop, int fixed_mode)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int active = 0, all_conv = 1, nonfinite = 0;
    for (int f = 0; f < nf; ++f) {
        if (ctl.frozen[f]) continue;
        const unsigned long long bits = ctl.res_bits[f];
        ctl.res_bits[f] = 0ull;
        const double r = __longlong_as_double((long long)bits);
        ctl.iters[f] += 1;
        ctl.resid[f] = r;
        ctl.parity[f] ^= 1;
        if (!(r <= 1.7976931348623157e308)) nonfinite = 1;
        const int conv = r <= delta_c;
        all_conv &= conv;
        ++active;
        if (per_bin_stop && conv && !fixed_mode) ctl.frozen[f] = 1;
    }
    if (!per_bin_stop && !fixed_mode && active > 0 && all_conv)
        for (int f = 0; f < nf; ++f) ctl.frozen[f] = 1;
    int stopped = 1;
    for (int f = 0; f < nf; ++f) stopped &= ctl.frozen[f] != 0;
    ctl.flags[0] = stopped;
    if (nonfinite) {
        ctl.flags[1] = 1;
        for (int f = 0; f < nf; ++f) ctl.frozen[f] = 1;
        ctl.flags[0] = 1;
    }
}

__global__ void flip_parity_kernel(int *parity, const int *frozen, int nf)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nf && !frozen[f]) parity[f] ^= 1;
}

__global__ void convert_f32_kernel(const double *src, float *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

__global__ void warm_start_kernel(const double *B, const double *eps, const double *J, double *S, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) S[i] = eps[i] * B[i] + (1.0 - eps[i]) * J[i];
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_sweep_stage_f64(const SweepArgs<double> &A, int waves, hipStream_t st)
{
    dim3 grid((unsigned)A.stage_cnt * 8u, (unsigned)A.nf);
    hipLaunchKernelGGL((sweep_stage_kernel<double, false>), grid, dim3(64 * waves), sweep_lds_bytes<double>(waves),
                       st, A);
    return hipGetLastError();
}

hipError_t launch_sweep_stage_f32(const SweepArgs<float> &A, int waves, hipStream_t st)
{
    dim3 grid((unsigned)A.stage_cnt * 8u, (unsigned)A.nf);
    hipLaunchKernelGGL((sweep_stage_kernel<float, true>), grid, dim3(64 * waves), sweep_lds_bytes<float>(waves),
                       st, A);
    return hipGetLastError();
}

hipError_t launch_lambda_star(const int n[3], const int bc_lo[3], const int bc_hi[3], int nf, int na,
                              const RayGeo *rays, const double *chi, double *lam, hipStream_t st)
{
    const int64_t tot = (int64_t)n[0] * n[1] * n[2] * nf;
    hipLaunchKernelGGL(lambda_star_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, st, n[0], n[1], n[2],
                       bc_lo[0], bc_hi[0], bc_lo[1], bc_hi[1], bc_lo[2], bc_hi[2], nf, na, rays, chi, lam);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_periodic_cold(const SweepArgs<Real> &A, hipStream_t st)
{
    for (int q = 0; q < 3; ++q) {
        if (!A.periodic[q]) continue;
        dim3 grid(blocks_for(A.plane[q], 256), (unsigned)A.na, (unsigned)A.nf);
        hipLaunchKernelGGL(periodic_cold_kernel<Real>, grid, dim3(256), 0, st, A, q);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
template hipError_t launch_periodic_cold<double>(const SweepArgs<double> &, hipStream_t);
template hipError_t launch_periodic_cold<float>(const SweepArgs<float> &, hipStream_t);

template <typename Real>
hipError_t launch_partial_sum(const Real *part, const double *S, int dform, int nf, int64_t cells,
                              const int *frozen, double *J, hipStream_t st)
{
    hipLaunchKernelGGL(partial_sum_kernel<Real>, dim3(blocks_for(cells * nf, 256)), dim3(256), 0, st, part, S,
                       dform, nf, cells, frozen, J);
    return hipGetLastError();
}
template hipError_t launch_partial_sum<double>(const double *, const double *, int, int, int64_t, const int *,
                                               double *, hipStream_t);
template hipError_t launch_partial_sum<float>(const float *, const double *, int, int, int64_t, const int *,
                                              double *, hipStream_t);

template <typename Real>
hipError_t launch_ali_update(const Real *part, int dform, int nf, int64_t cells, const double *B,
                             const double *eps, const double *lam, double *S64, float *S32, double *J,
                             AliCtl ctl, hipStream_t st)
{
    dim3 grid(blocks_for(cells, 256), (unsigned)nf);
    hipLaunchKernelGGL(ali_update_kernel<Real>, grid, dim3(256), 0, st, part, dform, nf, cells, B, eps, lam, S64,
                       S32, J, ctl);
    return hipGetLastError();
}
template hipError_t launch_ali_update<double>(const double *, int, int, int64_t, const double *, const double *,
                                              const double *, double *, float *, double *, AliCtl, hipStream_t);
template hipError_t launch_ali_update<float>(const float *, int, int, int64_t, const double *, const double *,
                                             const double *, double *, float *, double *, AliCtl, hipStream_t);

hipError_t launch_ali_finalize(AliCtl ctl, int nf, double delta_c, int per_bin_stop, int fixed_mode,
                               hipStream_t st)
{
    hipLaunchKernelGGL(ali_finalize_kernel, dim3(1), dim3(64), 0, st, ctl, nf, delta_c, per_bin_stop, fixed_mode);
    return hipGetLastError();
}

hipError_t launch_flip_parity(int *parity, const int *frozen, int nf, hipStream_t st)
{
    hipLaunchKernelGGL(flip_parity_kernel, dim3(blocks_for(nf, 64)), dim3(64), 0, st, parity, frozen, nf);
    return hipGetLastError();
}

hipError_t launch_convert_f32(const double *src, float *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(convert_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_warm_start(const double *B, const double *eps, const double *J, double *S, int64_t n,
                             hipStream_t st)
{
    hipLaunchKernelGGL(warm_start_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, B, eps, J, S, n);
    return hipGetLastError();
}

}  // namespace rtsc
