// Gauss-Seidel ALI (section 3.4) on gfx950: the backward half of an iteration.
//
// The paper takes the Gauss-Seidel scheme of Trujillo Bueno & Fabiani Bendicho (1995)
// and generalises it to 2D and 3D with bilinear interpolation: S is updated as soon
// as J is complete, and the short characteristics computed afterwards see the new
// value.  The blocks of the ordering here are the horizontal planes, from the top
// down.  The rays going up are swept first over the whole grid with the old S (the
// tile-wavefront kernel restricted to octants 0 .. 3): they depend only on vertices at
// or below their own plane, which are all still old when that plane is updated.  The
// rays going down then advance one plane per launch: launch t recomputes plane
// kn = nz - t from the final plane kn + 1 with the updated S of plane kn, and computes
// plane ko = nz - 1 - t from the final plane kn with the current (old) S of plane ko,
// which completes J on plane ko; the update of plane ko follows in its own launch.
//
// A ray going down that crosses a z face first ("steep") depends only on the plane
// above: a workgroup takes a 16 x 16 tile and recomputes plane kn on the tile plus
// one halo row and column on the upwind side, then plane ko on the tile.  A ray that
// crosses an x or y face first ("shallow", axis d) also depends on the previous
// vertex of its own plane along d, one vertex apart along the other in-plane axis e
// at most: it runs as a chain along d, one workgroup per ray and bin.  Per vertex
//   I_kn = E_n (w0 x + w1 y) + Q_n,   I_ko = E_o (w0 u + w1 v + w2 x + w3 y) + Q_o,
// with x, y (u, v) the chain's values on the previous column at e and at the upwind
// neighbour along e on plane kn (ko), and w the bilinear weights of the upwind face
// (along e, then z).  E and Q (the plane-above and source terms) do not depend on the
// chain: fifteen waves of the workgroup compute them for the next block of columns
// into LDS while wave 0 runs the recurrence over the current block; the values of the
// neighbour along e come from the next lane (a shuffle).  Ghost vertices (outside the
// grid) enter as constants: folded into Q above the grid, and as the starting column
// and the upwind neighbour of the lane at the grid's face along e.
//
// The FP32 path carries D = I - S (D0 = D- E + (S- - S0) g with S- - S0 formed in
// FP64); the periodic memory keeps I in FP64 in the layout of the sweep kernels (the
// flipped coordinates of each ray's octant).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rt_device.h"
#include "rt_internal.h"

namespace rtsc {
namespace {

constexpr int GT = kGsTile;
constexpr int GH = GT + 1;            // steep tile plus one vertex on the upwind side
constexpr int GHN = GH * GH;
constexpr int CHAIN_WAVES = 16;       // wave 0 runs the recurrence, the others fill blocks
constexpr int CHAIN_MAX_COLS = 16;

__device__ __forceinline__ int flip(int r, int sg, int n) { return sg > 0 ? r : n - 1 - r; }

template <typename Real>
__device__ __forceinline__ int64_t cell_of(const GsArgs<Real> &A, int f, int x, int y, int z)
{
    const int rx = fold(x, A.n[0], A.periodic[0]), ry = fold(y, A.n[1], A.periodic[1]);
    const int rz = fold(z, A.n[2], A.periodic[2]);
    return (int64_t)f * A.cells + ((int64_t)rz * A.n[1] + ry) * A.n[0] + rx;
}

// Intensity of ray `ray` (bin f) at a ghost vertex (x, y, z), one step outside the grid
// along one axis or more.  Outside a non-periodic face the face with the highest axis
// gives it: 0 (vacuum), B of the folded vertex (thermal) or the caller's incident
// intensity (fixed).  With only periodic axes outside it is the previous iteration's
// value at the wrapped vertex, kept on the ray's outgoing plane of the lowest such axis.
template <typename Real>
__device__ double ghost_I(const GsArgs<Real> &A, int f, int ray, int x, int y, int z)
{
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const bool ox = x < 0 || x >= nx, oy = y < 0 || y >= ny, oz = z < 0 || z >= nz;
    const int rx = fold(x, nx, A.periodic[0]), ry = fold(y, ny, A.periodic[1]), rz = fold(z, nz, A.periodic[2]);
    const int64_t cell = (int64_t)f * A.cells + ((int64_t)rz * ny + ry) * nx + rx;
    int q = -1, hi = 0;
    if (oz && !A.periodic[2]) {
        q = 2;
        hi = z >= nz;
    } else if (oy && !A.periodic[1]) {
        q = 1;
        hi = y >= ny;
    } else if (ox && !A.periodic[0]) {
        q = 0;
        hi = x >= nx;
    }
    if (q >= 0) {
        const int kind = hi ? A.bc_hi[q] : A.bc_lo[q];
        if (kind == BC_THERMAL) return A.B[cell];
        if (kind == BC_FIXED) {
            const double *F = A.fixed[2 * q + hi];
            const int64_t P = q == 0 ? (int64_t)ny * nz : (q == 1 ? (int64_t)nx * nz : (int64_t)nx * ny);
            const int64_t pidx = q == 0 ? (int64_t)rz * ny + ry : (q == 1 ? (int64_t)rz * nx + rx : (int64_t)ry * nx + rx);
            return F[((int64_t)f * A.na + A.rays[ray].gidx) * P + pidx];
        }
        return 0.0;
    }
    const int oct = A.rays[ray].oct;
    const int fx = flip(rx, (oct & 1) ? -1 : 1, nx), fy = flip(ry, (oct & 2) ? -1 : 1, ny);
    const int fz = flip(rz, (oct & 4) ? -1 : 1, nz);
    const int64_t rb = ((int64_t)f * A.na + ray) * 2 + A.parity[f];
    if (ox) return A.wrap[0][rb * ((int64_t)ny * nz) + (int64_t)fz * ny + fy];
    if (oy) return A.wrap[1][rb * ((int64_t)nx * nz) + (int64_t)fz * nx + fx];
    if (oz) return A.wrap[2][rb * ((int64_t)nx * ny) + (int64_t)fy * nx + fx];
    return 0.0;   // not a ghost vertex: no caller asks for one
}

// The value a sweep carries at a ghost vertex: I, or D = I - S of the folded vertex.
template <typename Real, bool DFORM>
__device__ __forceinline__ Real ghost_val(const GsArgs<Real> &A, int f, int ray, int x, int y, int z)
{
    const double I = ghost_I(A, f, ray, x, y, z);
    if constexpr (DFORM) return Real(I - A.S[cell_of(A, f, x, y, z)]);
    return Real(I);
}

// Segment of one vertex: attenuation E and source term c (plain: psim S- + psi0 S0;
// difference form: (S- - S0) g), from the interpolated chi- and S- and the vertex's own.
template <typename Real, bool DFORM>
__device__ __forceinline__ void segment(Real s_half, Real Cm, Real C0, double Sm, double S0, Real &E, Real &c)
{
    const Real dt = s_half * (Cm + C0);
    if constexpr (DFORM) {
        Real g;
        seg_coeffs(dt, E, g);
        c = Real(Sm - S0) * g;
    } else {
        Real pm, p0;
        seg_coeffs(dt, E, pm, p0);
        c = pm * Real(Sm) + p0 * Real(S0);
    }
}

// Store a final value of plane k on the ray's outgoing faces of the periodic in-plane
// axes (the next iteration's ghosts); I in FP64.
template <typename Real>
__device__ __forceinline__ void store_wrap(const GsArgs<Real> &A, int f, int ray, int x, int y, int z, double I)
{
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const int oct = A.rays[ray].oct;
    const int sx = (oct & 1) ? -1 : 1, sy = (oct & 2) ? -1 : 1, sz = (oct & 4) ? -1 : 1;
    const int64_t rb = ((int64_t)f * A.na + ray) * 2 + (A.parity[f] ^ 1);
    const int fx = flip(x, sx, nx), fy = flip(y, sy, ny), fz = flip(z, sz, nz);
    if (A.periodic[0] && fx == nx - 1) A.wrap[0][rb * ((int64_t)ny * nz) + (int64_t)fz * ny + fy] = I;
    if (A.periodic[1] && fy == ny - 1) A.wrap[1][rb * ((int64_t)nx * nz) + (int64_t)fz * nx + fx] = I;
}

// ---------------------------------------------------------------------------------
// Steep rays: one (ray, tile, bin) per workgroup of 256 lanes.
// ---------------------------------------------------------------------------------
template <typename Real, bool DFORM>
__global__ void __launch_bounds__(256) gs_steep_kernel(GsArgs<Real> A, int t)
{
    __shared__ Real Iw[GHN];
    __shared__ Real Cw[GHN];
    __shared__ double Sw[GHN];
    const int f = blockIdx.y;
    if (A.frozen[f]) return;
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const int kn = nz - t, ko = nz - 1 - t;
    const int di = A.ns + (int)blockIdx.x / A.ntiles;
    const int tile = (int)blockIdx.x % A.ntiles;
    const int ray = A.down[di];
    const RayGeo &G = A.rays[ray];
    const int sx = (G.oct & 1) ? -1 : 1, sy = (G.oct & 2) ? -1 : 1;
    const int x0 = (tile % A.tiles_x) * GT, y0 = (tile / A.tiles_x) * GT;
    // the halo lies one step upwind: x - sx, y - sy
    const int bx = x0 + (sx > 0 ? -1 : 0), by = y0 + (sy > 0 ? -1 : 0);
    const Real s_half = Real(0.5 * G.s);
    const Real w0 = Real(G.w4[0]), w1 = Real(G.w4[1]), w2 = Real(G.w4[2]), w3 = Real(G.w4[3]);
    const double w0d = G.w4[0], w1d = G.w4[1], w2d = G.w4[2], w3d = G.w4[3];
    const int64_t fc = (int64_t)f * A.cells;
    Real *plane_n = A.planes + (((int64_t)f * A.nd + di) * 2 + (kn & 1)) * A.pxy;
    const Real *plane_a = A.planes + (((int64_t)f * A.nd + di) * 2 + ((kn + 1) & 1)) * A.pxy;

    // plane kn on the tile and its halo: recomputed (t >= 1), or the top ghost plane
    for (int e = threadIdx.x; e < GHN; e += 256) {
        const int x = bx + e % GH, y = by + e / GH;
        if (x < -1 || x > nx || y < -1 || y > ny) {
            // more than one step outside the grid (a tile wider than the grid): no
            // vertex of the grid reads it
            Iw[e] = Real(0);
            Cw[e] = Real(0);
            Sw[e] = 0.0;
            continue;
        }
        const int64_t c = cell_of(A, f, x, y, kn);
        Real v;
        if (t == 0 || x < 0 || x >= nx || y < 0 || y >= ny) {
            v = ghost_val<Real, DFORM>(A, f, ray, x, y, kn);
        } else {
            Real Ia[4], Ca[4];
            double Sa[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int xa = x - ((q & 1) ? sx : 0), ya = y - ((q & 2) ? sy : 0);
                const bool in = kn + 1 < nz && xa >= 0 && xa < nx && ya >= 0 && ya < ny;
                const int64_t ca = cell_of(A, f, xa, ya, kn + 1);
                Ia[q] = in ? plane_a[(int64_t)ya * nx + xa] : ghost_val<Real, DFORM>(A, f, ray, xa, ya, kn + 1);
                Ca[q] = A.chi[ca];
                Sa[q] = A.S[ca];
            }
            const Real Im = w0 * Ia[0] + w1 * Ia[1] + w2 * Ia[2] + w3 * Ia[3];
            const Real Cm = w0 * Ca[0] + w1 * Ca[1] + w2 * Ca[2] + w3 * Ca[3];
            const double Sm = w0d * Sa[0] + w1d * Sa[1] + w2d * Sa[2] + w3d * Sa[3];
            Real E, cc;
            segment<Real, DFORM>(s_half, Cm, A.chi[c], Sm, A.S[c], E, cc);
            v = Im * E + cc;
            const bool own = x >= x0 && x < x0 + GT && y >= y0 && y < y0 + GT;
            if (own) {
                plane_n[(int64_t)y * nx + x] = v;
                store_wrap(A, f, ray, x, y, kn, DFORM ? double(v) + A.S[c] : double(v));
            }
        }
        Iw[e] = v;
        Cw[e] = A.chi[c];
        Sw[e] = A.S[c];
    }
    if (ko < 0) return;
    __syncthreads();
    // plane ko on the tile with the current S
    const int lx = threadIdx.x % GT, ly = threadIdx.x / GT;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= nx || y >= ny) return;
    const int hx = x - bx, hy = y - by;
    Real Ia[4], Ca[4];
    double Sa[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int h = (hy - ((q & 2) ? sy : 0)) * GH + (hx - ((q & 1) ? sx : 0));
        Ia[q] = Iw[h];
        Ca[q] = Cw[h];
        Sa[q] = Sw[h];
    }
    const int64_t c = fc + ((int64_t)ko * ny + y) * nx + x;
    const Real Im = w0 * Ia[0] + w1 * Ia[1] + w2 * Ia[2] + w3 * Ia[3];
    const Real Cm = w0 * Ca[0] + w1 * Ca[1] + w2 * Ca[2] + w3 * Ca[3];
    const double Sm = w0d * Sa[0] + w1d * Sa[1] + w2d * Sa[2] + w3d * Sa[3];
    Real E, cc;
    segment<Real, DFORM>(s_half, Cm, A.chi[c], Sm, A.S[c], E, cc);
    const Real v = Im * E + cc;
    A.part[((int64_t)di * A.nf + f) * A.pxy + (int64_t)y * nx + x] = Real(G.wk) * v;
}

// ---------------------------------------------------------------------------------
// Shallow rays: one chain (ray, bin) per workgroup of CHAIN_WAVES waves.
// ---------------------------------------------------------------------------------
template <typename Real>
struct Chain {
    int f, di, ray, d, sd, se, Nd, Ne, nep, cols, t, kn, ko;
    Real w0, w1, w2, w3, s_half, wk;
    double w0d, w1d, w2d, w3d;
    // LDS, per buffer: [4][cols][nep] coefficients E_n, Q_n, E_o, Q_o; [cols][nep] S of
    // plane kn (the difference form's periodic memory keeps I = D + S); [cols] ghost
    // neighbours along e of the boundary lane on planes kn and ko
    double *s0[2];
    Real *coef[2];
    Real *gy[2], *gv[2];
    Real *x0, *u0;   // [nep] the column before the first (ghosts) on planes kn and ko
};

template <typename Real>
__device__ __forceinline__ void chain_xy(const Chain<Real> &C, int pd, int pe, int &x, int &y)
{
    x = C.d == 0 ? pd : pe;
    y = C.d == 0 ? pe : pd;
}

// Coefficients of the columns c0 .. c0 + cols - 1 into buffer `buf`.
template <typename Real, bool DFORM>
__device__ void chain_fill(const GsArgs<Real> &A, const Chain<Real> &C, int buf, int c0, int tid, int nthr)
{
    const int nz = A.n[2];
    const int kn = C.kn, ko = C.ko;
    const int64_t slot = (int64_t)C.cols * C.nep;
    Real *cf = C.coef[buf];
    const Real *above = A.planes + (((int64_t)C.f * A.nd + C.di) * 2 + ((kn + 1) & 1)) * A.pxy;
    for (int it = tid; it < C.cols * C.nep; it += nthr) {
        const int cc = it / C.nep, pe = it - cc * C.nep;
        const int c = c0 + cc;
        Real En = Real(0), Qn = Real(0), Eo = Real(0), Qo = Real(0);
        double s0 = 0.0;
        if (c < C.Nd && pe < C.Ne) {
            const int pd = C.sd > 0 ? c : C.Nd - 1 - c;
            const int ud = pd - C.sd, ue = pe - C.se;
            int x, y, xu, yu, xv, yv;
            chain_xy(C, pd, pe, x, y);
            chain_xy(C, ud, pe, xu, yu);
            chain_xy(C, ud, ue, xv, yv);
            const int64_t cu = cell_of(A, C.f, xu, yu, kn), cv = cell_of(A, C.f, xv, yv, kn);
            if (C.t == 0) {
                // the plane above the grid stands in for plane kn
                Qn = ghost_val<Real, DFORM>(A, C.f, C.ray, x, y, nz);
            } else {
                // upwind face corners along (e, z): (0, 0) (1, 0) in plane kn, (0, 1) (1, 1) above
                const int64_t cu1 = cell_of(A, C.f, xu, yu, kn + 1), cv1 = cell_of(A, C.f, xv, yv, kn + 1);
                const int64_t c0v = cell_of(A, C.f, x, y, kn);
                const bool in_u = kn + 1 < nz && ud >= 0 && ud < C.Nd;
                const bool in_v = in_u && ue >= 0 && ue < C.Ne;
                const Real Iu1 = in_u ? above[(int64_t)ud * C.Ne + pe] : ghost_val<Real, DFORM>(A, C.f, C.ray, xu, yu, kn + 1);
                const Real Iv1 = in_v ? above[(int64_t)ud * C.Ne + ue] : ghost_val<Real, DFORM>(A, C.f, C.ray, xv, yv, kn + 1);
                const Real Cm = C.w0 * A.chi[cu] + C.w1 * A.chi[cv] + C.w2 * A.chi[cu1] + C.w3 * A.chi[cv1];
                const double Sm = C.w0d * A.S[cu] + C.w1d * A.S[cv] + C.w2d * A.S[cu1] + C.w3d * A.S[cv1];
                Real E, src;
                segment<Real, DFORM>(C.s_half, Cm, A.chi[c0v], Sm, A.S[c0v], E, src);
                En = E;
                Qn = E * (C.w2 * Iu1 + C.w3 * Iv1) + src;
                s0 = A.S[c0v];
            }
            if (ko >= 0) {
                const int64_t du = cell_of(A, C.f, xu, yu, ko), dv = cell_of(A, C.f, xv, yv, ko);
                const int64_t c0o = cell_of(A, C.f, x, y, ko);
                const Real Cm = C.w0 * A.chi[du] + C.w1 * A.chi[dv] + C.w2 * A.chi[cu] + C.w3 * A.chi[cv];
                const double Sm = C.w0d * A.S[du] + C.w1d * A.S[dv] + C.w2d * A.S[cu] + C.w3d * A.S[cv];
                segment<Real, DFORM>(C.s_half, Cm, A.chi[c0o], Sm, A.S[c0o], Eo, Qo);
            }
        }
        cf[0 * slot + it] = En;
        cf[1 * slot + it] = Qn;
        cf[2 * slot + it] = Eo;
        cf[3 * slot + it] = Qo;
        if constexpr (DFORM) C.s0[buf][it] = s0;
    }
    // the boundary lane's upwind neighbour along e lies outside the grid
    for (int cc = tid; cc < C.cols; cc += nthr) {
        const int c = c0 + cc;
        Real gy = Real(0), gv = Real(0);
        if (c < C.Nd) {
            const int pd = C.sd > 0 ? c : C.Nd - 1 - c;
            const int pb = C.se > 0 ? 0 : C.Ne - 1;
            int xv, yv;
            chain_xy(C, pd - C.sd, pb - C.se, xv, yv);
            gy = ghost_val<Real, DFORM>(A, C.f, C.ray, xv, yv, kn);
            if (ko >= 0) gv = ghost_val<Real, DFORM>(A, C.f, C.ray, xv, yv, ko);
        }
        C.gy[buf][cc] = gy;
        C.gv[buf][cc] = gv;
    }
}

template <typename Real, bool DFORM, int M>
__global__ void __launch_bounds__(64 * CHAIN_WAVES) gs_chain_kernel(GsArgs<Real> A, int t, int cols)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int f = blockIdx.y;
    if (A.frozen[f]) return;
    Chain<Real> C;
    C.f = f;
    C.di = blockIdx.x;
    C.ray = A.down[C.di];
    const RayGeo &G = A.rays[C.ray];
    C.d = G.d;
    const int e = 1 - C.d;
    C.sd = (G.oct >> C.d) & 1 ? -1 : 1;
    C.se = (G.oct >> e) & 1 ? -1 : 1;
    C.Nd = A.n[C.d];
    C.Ne = A.n[e];
    C.nep = 64 * M;
    C.cols = cols;
    C.t = t;
    C.kn = A.n[2] - t;
    C.ko = A.n[2] - 1 - t;
    C.w0 = Real(G.w4[0]);
    C.w1 = Real(G.w4[1]);
    C.w2 = Real(G.w4[2]);
    C.w3 = Real(G.w4[3]);
    C.w0d = G.w4[0];
    C.w1d = G.w4[1];
    C.w2d = G.w4[2];
    C.w3d = G.w4[3];
    C.s_half = Real(0.5 * G.s);
    C.wk = Real(G.wk);
    {
        const int64_t slot = (int64_t)cols * C.nep;
        unsigned char *p = lds_raw;
        for (int b = 0; b < 2; ++b) {
            C.s0[b] = reinterpret_cast<double *>(p);
            p += DFORM ? slot * sizeof(double) : 0;
        }
        for (int b = 0; b < 2; ++b) {
            C.coef[b] = reinterpret_cast<Real *>(p);
            p += 4 * slot * sizeof(Real);
        }
        for (int b = 0; b < 2; ++b) {
            C.gy[b] = reinterpret_cast<Real *>(p);
            p += cols * sizeof(Real);
            C.gv[b] = reinterpret_cast<Real *>(p);
            p += cols * sizeof(Real);
        }
        C.x0 = reinterpret_cast<Real *>(p);
        p += C.nep * sizeof(Real);
        C.u0 = reinterpret_cast<Real *>(p);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    // prologue: block 0 and the column before the first
    chain_fill<Real, DFORM>(A, C, 0, 0, threadIdx.x, blockDim.x);
    for (int pe = threadIdx.x; pe < C.nep; pe += blockDim.x) {
        Real x0 = Real(0), u0 = Real(0);
        if (pe < C.Ne) {
            const int ud = C.sd > 0 ? -1 : C.Nd;
            int x, y;
            chain_xy(C, ud, pe, x, y);
            x0 = ghost_val<Real, DFORM>(A, f, C.ray, x, y, C.kn);
            if (C.ko >= 0) u0 = ghost_val<Real, DFORM>(A, f, C.ray, x, y, C.ko);
        }
        C.x0[pe] = x0;
        C.u0[pe] = u0;
    }
    __syncthreads();

    Real xr[M], ur[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        xr[m] = C.x0[lane * M + m];
        ur[m] = C.u0[lane * M + m];
    }
    Real *plane_n = A.planes + (((int64_t)f * A.nd + C.di) * 2 + (C.kn & 1)) * A.pxy;
    Real *part = A.part + ((int64_t)C.di * A.nf + f) * A.pxy;
    const int nb = (C.Nd + cols - 1) / cols;
    const int64_t slot = (int64_t)cols * C.nep;
    for (int b = 0; b < nb; ++b) {
        if (wave == 0) {
            const int buf = b & 1;
            const Real *cf = C.coef[buf];
            for (int cc = 0; cc < cols; ++cc) {
                const int c = b * cols + cc;
                if (c >= C.Nd) break;   // uniform over the wave
                const int pd = C.sd > 0 ? c : C.Nd - 1 - c;
                const Real gy = C.gy[buf][cc], gv = C.gv[buf][cc];
                // neighbours along e from the next lane: its first (se < 0) or last
                // (se > 0) value
                const Real sx = C.se > 0 ? __shfl_up(xr[M - 1], 1) : __shfl_down(xr[0], 1);
                const Real su = C.se > 0 ? __shfl_up(ur[M - 1], 1) : __shfl_down(ur[0], 1);
                Real xn[M], un[M];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int pe = lane * M + m;
                    Real y, v;
                    if (C.se > 0) {
                        y = m > 0 ? xr[m - 1] : sx;
                        v = m > 0 ? ur[m - 1] : su;
                        if (pe == 0) {
                            y = gy;
                            v = gv;
                        }
                    } else {
                        y = m < M - 1 ? xr[m + 1] : sx;
                        v = m < M - 1 ? ur[m + 1] : su;
                        if (pe == C.Ne - 1) {
                            y = gy;
                            v = gv;
                        }
                    }
                    const int o = cc * C.nep + pe;
                    const Real En = cf[o], Qn = cf[slot + o], Eo = cf[2 * slot + o], Qo = cf[3 * slot + o];
                    xn[m] = En * (C.w0 * xr[m] + C.w1 * y) + Qn;
                    un[m] = Eo * (C.w0 * ur[m] + C.w1 * v + C.w2 * xr[m] + C.w3 * y) + Qo;
                }
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int pe = lane * M + m;
                    if (pe < C.Ne) {
                        const int64_t o = (int64_t)pd * C.Ne + pe;
                        if (t > 0) {
                            plane_n[o] = xn[m];
                            int x, y;
                            chain_xy(C, pd, pe, x, y);
                            double I = double(xn[m]);
                            if constexpr (DFORM) I += C.s0[buf][cc * C.nep + pe];
                            store_wrap(A, f, C.ray, x, y, C.kn, I);
                        }
                        if (C.ko >= 0) part[o] = C.wk * un[m];
                    }
                    xr[m] = xn[m];
                    ur[m] = un[m];
                }
            }
        } else if (b + 1 < nb) {
            chain_fill<Real, DFORM>(A, C, (b + 1) & 1, (b + 1) * cols, threadIdx.x - 64, blockDim.x - 64);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------
// Update of plane k (eq. dsjacobi) once its J is complete.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_max_bits(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o > v ? o : v;
    }
    return v;
}

template <typename Real, bool DFORM>
__global__ void __launch_bounds__(256) gs_update_kernel(GsArgs<Real> A, int k)
{
    __shared__ unsigned long long red[4];
    const int f = blockIdx.y;
    if (A.frozen[f]) return;
    const int nx = A.n[0], ny = A.n[1];
    const int64_t stride_up = (int64_t)A.nf * A.cells;
    unsigned long long rb = 0ull;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < A.pxy; p += (int64_t)gridDim.x * 256) {
        const int x = (int)(p % nx), y = (int)(p / nx);
        const int64_t i = (int64_t)f * A.cells + (int64_t)k * A.pxy + p;
        double sum = 0.0;
#pragma unroll
        for (int o = 0; o < 4; ++o) sum += (double)A.part_up[o * stride_up + i];
        for (int di = 0; di < A.nd; ++di) {
            // chains along x keep the plane with y fastest
            const int64_t idx = A.rays[A.down[di]].d == 0 ? (int64_t)x * ny + y : p;
            sum += (double)A.part[((int64_t)di * A.nf + f) * A.pxy + idx];
        }
        const double S = A.S[i], e = A.eps[i];
        double num;
        if constexpr (DFORM) {
            num = (1.0 - e) * sum + e * (A.B[i] - S);
            A.J[i] = S + sum;
        } else {
            num = (1.0 - e) * sum + e * A.B[i] - S;
            A.J[i] = sum;
        }
        const double dS = num / (1.0 - (1.0 - e) * A.lam[i]);
        const double Sn = S + dS;
        A.S[i] = Sn;
        const double r = (Sn != 0.0) ? fabs(dS) / fabs(Sn) : 0.0;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(r);
        rb = bits > rb ? bits : rb;
    }
    rb = wave_max_bits(rb);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rb;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int w = 1; w < 4; ++w) m = red[w] > m ? red[w] : m;
        const int64_t slot = ((int64_t)k * gridDim.x + blockIdx.x) % A.nblk;
        atomicMax(A.blockmax + (int64_t)f * A.nblk + slot, m);
    }
}

__global__ void gs_clear_kernel(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Dynamic LDS of a chain workgroup with `cols` columns per block.
template <typename Real, bool DFORM>
size_t chain_lds(int nep, int cols)
{
    const size_t slot = (size_t)cols * nep;
    return 2 * ((DFORM ? slot * sizeof(double) : 0) + 4 * slot * sizeof(Real) + 2 * cols * sizeof(Real)) +
           2 * (size_t)nep * sizeof(Real);
}

template <typename Real, bool DFORM>
int chain_cols(int nep)
{
    int cols = CHAIN_MAX_COLS;
    while (cols > 1 && chain_lds<Real, DFORM>(nep, cols) > 64 * 1024) --cols;
    return cols;
}

template <typename Real, bool DFORM, int M>
void launch_chain(const GsArgs<Real> &A, int t, hipStream_t st)
{
    const int cols = chain_cols<Real, DFORM>(64 * M);
    const size_t lds = chain_lds<Real, DFORM>(64 * M, cols);
    hipLaunchKernelGGL((gs_chain_kernel<Real, DFORM, M>), dim3((unsigned)A.ns, (unsigned)A.nf),
                       dim3(64 * CHAIN_WAVES), lds, st, A, t, cols);
}

}  // namespace

template <typename Real>
hipError_t launch_gs_plane(const GsArgs<Real> &A, int t, hipStream_t st)
{
    constexpr bool DF = sizeof(Real) == 4;
    if (A.nd > A.ns)
        hipLaunchKernelGGL((gs_steep_kernel<Real, DF>), dim3((unsigned)((A.nd - A.ns) * A.ntiles), (unsigned)A.nf),
                           dim3(256), 0, st, A, t);
    if (A.ns > 0) {
        const int ne = std::max(A.n[0], A.n[1]);
        if (ne <= 64)
            launch_chain<Real, DF, 1>(A, t, st);
        else if (ne <= 128)
            launch_chain<Real, DF, 2>(A, t, st);
        else
            launch_chain<Real, DF, 4>(A, t, st);
    }
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_gs_update(const GsArgs<Real> &A, int k, hipStream_t st)
{
    constexpr bool DF = sizeof(Real) == 4;
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>(64, (A.pxy + 2047) / 2048));
    hipLaunchKernelGGL((gs_update_kernel<Real, DF>), dim3((unsigned)per, (unsigned)A.nf), dim3(256), 0, st, A, k);
    return hipGetLastError();
}

hipError_t launch_gs_clear(unsigned long long *blockmax, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(gs_clear_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, blockmax, n);
    return hipGetLastError();
}

template hipError_t launch_gs_plane<float>(const GsArgs<float> &, int, hipStream_t);
template hipError_t launch_gs_plane<double>(const GsArgs<double> &, int, hipStream_t);
template hipError_t launch_gs_update<float>(const GsArgs<float> &, int, hipStream_t);
template hipError_t launch_gs_update<double>(const GsArgs<double> &, int, hipStream_t);

}  // namespace rtsc
