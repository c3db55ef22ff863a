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
// at most: it runs as a chain along d, one wave per ray and bin.  Per vertex
//   I_kn = E_n (w0 x + w1 y) + Q_n,   I_ko = E_o (w0 u + w1 v + w2 x + w3 y) + Q_o,
// with x, y (u, v) the chain's values on the previous column at e and at the upwind
// neighbour along e on plane kn (ko), and w the bilinear weights of the upwind face
// (along e, then z).  E and Q (the plane-above and source terms) do not depend on the
// chain: they are computed for every vertex of every chain in parallel, in the launch
// of the steep tiles, and the chain's wave streams them a few columns ahead of its
// step; the values of the neighbour along e come from the next lane (a shuffle).
// Ghost vertices (outside the grid) enter as constants: folded into Q above the grid,
// and as the starting column and the upwind neighbour of the lane at the grid's face
// along e.
//
// The FP32 path carries D = I - S (D0 = D- E + (S- - S0) g with S- - S0 formed in
// FP64); the periodic memory keeps I in FP64 in the layout of the sweep kernels (the
// flipped coordinates of each ray's octant).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "rt_device.h"
#include "rt_internal.h"

namespace rtsc {
namespace {

constexpr int GT = kGsTile;
constexpr int GH = GT + 1;            // steep tile plus one vertex on the upwind side
constexpr int GHN = GH * GH;

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
__device__ __forceinline__ void steep_tile(const GsArgs<Real> &A, int f, int item, int t)
{
    __shared__ Real Iw[GHN];
    __shared__ Real Cw[GHN];
    __shared__ double Sw[GHN];
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const int kn = nz - t, ko = nz - 1 - t;
    const int di = A.ns + item / A.ntiles;
    const int tile = item % A.ntiles;
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
// Shallow rays.  The coefficients of every vertex of planes kn and ko of every chain
// are computed in parallel (with the steep tiles, in one launch); one wave per chain
// then runs the recurrence, lanes along e, streaming the coefficients a few columns
// ahead of the step.
// ---------------------------------------------------------------------------------
template <typename Real>
struct Chain {
    int f, di, ray, d, e, sd, se, Nd, Ne, kn, ko;
};

template <typename Real>
__device__ __forceinline__ Chain<Real> chain_of(const GsArgs<Real> &A, int f, int di, int t)
{
    Chain<Real> C;
    C.f = f;
    C.di = di;
    C.ray = A.down[di];
    const RayGeo &G = A.rays[C.ray];
    C.d = G.d;
    C.e = 1 - C.d;
    C.sd = (G.oct >> C.d) & 1 ? -1 : 1;
    C.se = (G.oct >> C.e) & 1 ? -1 : 1;
    C.Nd = A.n[C.d];
    C.Ne = A.n[C.e];
    C.kn = A.n[2] - t;
    C.ko = A.n[2] - 1 - t;
    return C;
}

template <typename Real>
__device__ __forceinline__ void chain_xy(const Chain<Real> &C, int pd, int pe, int &x, int &y)
{
    x = C.d == 0 ? pd : pe;
    y = C.d == 0 ? pe : pd;
}

// Index of (pd, pe, z) in the chain's own ordering of chi and S: [z][pd][pe], which is
// the grid layout for chains along y and the y-fastest copy for chains along x.  pd
// and pe may be one step outside (folded like any ghost vertex); z is clamped.
template <typename Real>
__device__ __forceinline__ int64_t ch_idx(const GsArgs<Real> &A, const Chain<Real> &C, int pd, int pe, int z)
{
    const int fd = fold(pd, C.Nd, A.periodic[C.d]), fe = fold(pe, C.Ne, A.periodic[C.e]);
    const int fz = z < A.n[2] ? z : A.n[2] - 1;
    return (int64_t)C.f * A.cells + ((int64_t)fz * C.Nd + fd) * C.Ne + fe;
}

// Coefficients of one vertex (pd, pe) of a chain, chain layout o = pd Ne + pe:
// E_n, Q_n (plane kn), E_o, Q_o (plane ko).  The vertex in the first column (pd = 0)
// also writes the column before the first (ghosts) at its pe; the vertex at pe = 0
// writes the ghost neighbours along e of the boundary lane for its column.
template <typename Real, bool DFORM>
__device__ __forceinline__ void chain_coef(const GsArgs<Real> &A, const Chain<Real> &C, int64_t v, int t)
{
    const int nz = A.n[2];
    const int kn = C.kn, ko = C.ko;
    const RayGeo &G = A.rays[C.ray];
    const Real s_half = Real(0.5 * G.s);
    const Real w0 = Real(G.w4[0]), w1 = Real(G.w4[1]), w2 = Real(G.w4[2]), w3 = Real(G.w4[3]);
    const double w0d = G.w4[0], w1d = G.w4[1], w2d = G.w4[2], w3d = G.w4[3];
    const Real *chi = C.d == 0 ? A.chi_t : A.chi;
    const double *S = C.d == 0 ? A.S_t : A.S;
    const int pd = (int)(v / C.Ne), pe = (int)(v - (int64_t)pd * C.Ne);
    const int ud = pd - C.sd, ue = pe - C.se;
    Real En = Real(0), Qn = Real(0), Eo = Real(0), Qo = Real(0);
    if (t == 0) {
        // the plane above the grid stands in for plane kn
        int x, y;
        chain_xy(C, pd, pe, x, y);
        Qn = ghost_val<Real, DFORM>(A, C.f, C.ray, x, y, nz);
    } else {
        // upwind face corners along (e, z): (0, 0) (1, 0) in plane kn, (0, 1) (1, 1) above
        const Real *above = A.planes + (((int64_t)C.f * A.nd + C.di) * 2 + ((kn + 1) & 1)) * A.pxy;
        const int64_t cu = ch_idx(A, C, ud, pe, kn), cv = ch_idx(A, C, ud, ue, kn);
        const int64_t cu1 = ch_idx(A, C, ud, pe, kn + 1), cv1 = ch_idx(A, C, ud, ue, kn + 1);
        const int64_t c0v = ch_idx(A, C, pd, pe, kn);
        const bool in_u = kn + 1 < nz && ud >= 0 && ud < C.Nd;
        const bool in_v = in_u && ue >= 0 && ue < C.Ne;
        Real Iu1, Iv1;
        if (in_v) {
            Iu1 = above[(int64_t)ud * C.Ne + pe];
            Iv1 = above[(int64_t)ud * C.Ne + ue];
        } else {
            int xu, yu, xv, yv;
            chain_xy(C, ud, pe, xu, yu);
            chain_xy(C, ud, ue, xv, yv);
            Iu1 = in_u ? above[(int64_t)ud * C.Ne + pe] : ghost_val<Real, DFORM>(A, C.f, C.ray, xu, yu, kn + 1);
            Iv1 = ghost_val<Real, DFORM>(A, C.f, C.ray, xv, yv, kn + 1);
        }
        const Real Cm = w0 * chi[cu] + w1 * chi[cv] + w2 * chi[cu1] + w3 * chi[cv1];
        const double Sm = w0d * S[cu] + w1d * S[cv] + w2d * S[cu1] + w3d * S[cv1];
        Real E, src;
        segment<Real, DFORM>(s_half, Cm, chi[c0v], Sm, S[c0v], E, src);
        En = E;
        Qn = E * (w2 * Iu1 + w3 * Iv1) + src;
    }
    if (ko >= 0) {
        const int64_t du = ch_idx(A, C, ud, pe, ko), dv = ch_idx(A, C, ud, ue, ko);
        const int64_t cu = ch_idx(A, C, ud, pe, ko + 1), cv = ch_idx(A, C, ud, ue, ko + 1);
        const int64_t c0o = ch_idx(A, C, pd, pe, ko);
        const Real Cm = w0 * chi[du] + w1 * chi[dv] + w2 * chi[cu] + w3 * chi[cv];
        const double Sm = w0d * S[du] + w1d * S[dv] + w2d * S[cu] + w3d * S[cv];
        segment<Real, DFORM>(s_half, Cm, chi[c0o], Sm, S[c0o], Eo, Qo);
    }
    Real *cf = A.coef + (((int64_t)C.f * A.ns + C.di) * A.pxy + v) * 4;
    cf[0] = En;
    cf[1] = Qn;
    cf[2] = Eo;
    cf[3] = Qo;
    Real *gh = A.gh + ((int64_t)C.f * A.ns + C.di) * 4 * A.nmax;
    if (DFORM && t > 0) {
        // S where the chain writes the periodic memory (I = D + S): the outgoing face
        // along e (per column) and the last column (per pe)
        const int64_t c0v = ch_idx(A, C, pd, pe, kn);
        const double *S = C.d == 0 ? A.S_t : A.S;
        if (pe == (C.se > 0 ? C.Ne - 1 : 0)) reinterpret_cast<double *>(A.ghS)[((int64_t)C.f * A.ns + C.di) * 2 * A.nmax + pd] = S[c0v];
        if (pd == (C.sd > 0 ? C.Nd - 1 : 0)) reinterpret_cast<double *>(A.ghS)[((int64_t)C.f * A.ns + C.di) * 2 * A.nmax + A.nmax + pe] = S[c0v];
    }
    if (pe == 0) {
        // the boundary lane's upwind neighbour along e lies outside the grid
        const int pb = C.se > 0 ? 0 : C.Ne - 1;
        int xv, yv;
        chain_xy(C, ud, pb - C.se, xv, yv);
        gh[pd] = ghost_val<Real, DFORM>(A, C.f, C.ray, xv, yv, kn);
        gh[A.nmax + pd] = ko >= 0 ? ghost_val<Real, DFORM>(A, C.f, C.ray, xv, yv, ko) : Real(0);
    }
    if (pd == 0) {
        // the column before the first along d
        int x, y;
        chain_xy(C, C.sd > 0 ? -1 : C.Nd, pe, x, y);
        gh[2 * A.nmax + pe] = ghost_val<Real, DFORM>(A, C.f, C.ray, x, y, kn);
        gh[3 * A.nmax + pe] = ko >= 0 ? ghost_val<Real, DFORM>(A, C.f, C.ray, x, y, ko) : Real(0);
    }
}

// Launch t, first part: the steep tiles, then the chain coefficients.
template <typename Real, bool DFORM>
__global__ void __launch_bounds__(256) gs_prep_kernel(GsArgs<Real> A, int t)
{
    const int f = blockIdx.y;
    if (A.frozen[f]) return;
    if ((int)blockIdx.x < A.steep_blocks) {
        if ((int)blockIdx.x < (A.nd - A.ns) * A.ntiles) steep_tile<Real, DFORM>(A, f, blockIdx.x, t);
        return;
    }
    // Workgroups are dealt to the 8 XCDs in turn: coefficient block j goes to XCD
    // j % 8 (steep_blocks is a multiple of 8), and serves a chain di with di % 8 equal
    // to it, whose wave (block di of the chain launch) runs on the same XCD and reads
    // the coefficients from that XCD's L2.
    const int j = (int)blockIdx.x - A.steep_blocks;
    const int q = j & 7, r = j >> 3;
    const int cb = (int)((A.pxy + 255) / 256);            // blocks per chain
    const int di = q + 8 * (r / cb);
    if (di >= A.ns) return;
    const int64_t v = (int64_t)(r % cb) * 256 + threadIdx.x;
    if (v >= A.pxy) return;
    chain_coef<Real, DFORM>(A, chain_of(A, f, di, t), v, t);
}

// Launch t, second part: one wave per chain (ray, bin).  Lane l holds the M vertices
// pe = l M .. l M + M - 1 of the current column; the upwind neighbour along e of the
// first (se > 0) or last (se < 0) of them is in the next lane.  The columns are taken
// in groups of P: the coefficients of the next group are loaded at the start of a
// group, so the wait for them at the group's end finds loads issued P steps before.
// NEW: plane kn is recomputed (t > 0); OLD: plane ko is computed (t < nz); FULL: every
// lane holds M vertices of the column (Ne = 64 M).  The periodic memory of plane kn is
// written after the recurrence: the outgoing face along e from the plane just written,
// the last column from the registers.
template <typename Real, bool DFORM, int M, bool NEW, bool OLD, bool FULL>
__global__ void __launch_bounds__(64) gs_chain_kernel(GsArgs<Real> A, int t)
{
    constexpr int P = (sizeof(Real) == 4 ? 16 : 8) / M;
    const int f = blockIdx.y;
    if (A.frozen[f]) return;
    const Chain<Real> C = chain_of(A, f, blockIdx.x, t);
    const RayGeo &G = A.rays[C.ray];
    const Real w0 = Real(G.w4[0]), w1 = Real(G.w4[1]), w2 = Real(G.w4[2]), w3 = Real(G.w4[3]);
    const Real wk = Real(G.wk);
    const int lane = threadIdx.x;
    const Real *cf = A.coef + ((int64_t)f * A.ns + C.di) * A.pxy * 4;
    const Real *gh = A.gh + ((int64_t)f * A.ns + C.di) * 4 * A.nmax;
    const double *ghS = reinterpret_cast<const double *>(A.ghS) + ((int64_t)f * A.ns + C.di) * 2 * A.nmax;
    Real *plane_n = A.planes + (((int64_t)f * A.nd + C.di) * 2 + (C.kn & 1)) * A.pxy;
    Real *part = A.part + ((int64_t)C.di * A.nf + f) * A.pxy;
    int pe_m[M];
    bool ok_m[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        pe_m[m] = lane * M + m;
        ok_m[m] = FULL || pe_m[m] < C.Ne;
    }
    // the lane holding the neighbour of this lane's boundary vertex, and which vertex
    const int src = C.se > 0 ? lane - 1 : lane + 1;
    const bool first_is_nb = C.se < 0;   // the next lane's first vertex (se < 0) or last
    const int pe_edge = C.se > 0 ? 0 : C.Ne - 1;   // the vertex whose neighbour is a ghost
    Real xr[M], ur[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int pe = ok_m[m] ? pe_m[m] : 0;
        xr[m] = ok_m[m] ? gh[2 * A.nmax + pe] : Real(0);
        ur[m] = ok_m[m] ? gh[3 * A.nmax + pe] : Real(0);
    }
    // ghost neighbours of the boundary lane per column, staged in LDS
    __shared__ Real s_gy[kGsMaxLanes], s_gv[kGsMaxLanes];
    for (int k = lane; k < C.Nd; k += 64) {
        s_gy[k] = gh[k];
        s_gv[k] = gh[A.nmax + k];
    }
    __syncthreads();
    Real aEn[P][M], aQn[P][M], aEo[P][M], aQo[P][M];
    Real bEn[P][M], bQn[P][M], bEo[P][M], bQo[P][M];
    const int64_t dstep = C.sd > 0 ? C.Ne : -(int64_t)C.Ne;      // chain offset per column
    const int64_t o0 = C.sd > 0 ? 0 : (int64_t)(C.Nd - 1) * C.Ne;  // column c = 0
    auto fetch = [&](int c, Real (&En)[M], Real (&Qn)[M], Real (&Eo)[M], Real (&Qo)[M]) {
        const int cc = c < C.Nd ? c : C.Nd - 1;      // past the end: any valid column
        const int64_t ob = o0 + cc * dstep;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int64_t o = ob + (ok_m[m] ? pe_m[m] : 0);
            if constexpr (sizeof(Real) == 4) {
                const float4 q4 = *reinterpret_cast<const float4 *>(cf + o * 4);
                En[m] = q4.x;
                Qn[m] = q4.y;
                Eo[m] = q4.z;
                Qo[m] = q4.w;
            } else {
                const double2 a2 = *reinterpret_cast<const double2 *>(cf + o * 4);
                const double2 b2 = *reinterpret_cast<const double2 *>(cf + o * 4 + 2);
                En[m] = a2.x;
                Qn[m] = a2.y;
                Eo[m] = b2.x;
                Qo[m] = b2.y;
            }
        }
    };
#pragma unroll
    for (int j = 0; j < P; ++j) fetch(j, aEn[j], aQn[j], aEo[j], aQo[j]);
    for (int c0 = 0; c0 < C.Nd; c0 += P) {
        // the next group's coefficients first
#pragma unroll
        for (int j = 0; j < P; ++j) fetch(c0 + P + j, bEn[j], bQn[j], bEo[j], bQo[j]);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int c = c0 + j;
            const int cc = c < C.Nd ? c : C.Nd - 1;
            const int pd = C.sd > 0 ? cc : C.Nd - 1 - cc;
            const Real gy = s_gy[pd], gv = OLD ? s_gv[pd] : Real(0);
            // the neighbour along e of this lane's boundary vertex, from the next lane
            const Real sx = __shfl(first_is_nb ? xr[0] : xr[M - 1], src);
            Real su = Real(0);
            if constexpr (OLD) su = __shfl(first_is_nb ? ur[0] : ur[M - 1], src);
            Real xn[M], un[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                Real y, v = Real(0);
                if (M == 1) {
                    y = sx;
                    v = su;
                } else if (m == 0) {
                    y = first_is_nb ? xr[1] : sx;
                    if constexpr (OLD) v = first_is_nb ? ur[1] : su;
                } else if (m == M - 1) {
                    y = first_is_nb ? sx : xr[M - 2];
                    if constexpr (OLD) v = first_is_nb ? su : ur[M - 2];
                } else {
                    y = first_is_nb ? xr[m + 1] : xr[m - 1];
                    if constexpr (OLD) v = first_is_nb ? ur[m + 1] : ur[m - 1];
                }
                // the vertex at the grid's face along e takes the ghost neighbour
                const bool edge = pe_m[m] == pe_edge;
                y = edge ? gy : y;
                xn[m] = aEn[j][m] * (w0 * xr[m] + w1 * y) + aQn[j][m];
                if constexpr (OLD) {
                    v = edge ? gv : v;
                    un[m] = aEo[j][m] * (w0 * ur[m] + w1 * v + w2 * xr[m] + w3 * y) + aQo[j][m];
                }
            }
            if (c < C.Nd) {   // uniform over the wave; past the end nothing is kept
                const int64_t ob = o0 + c * dstep;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (!ok_m[m]) continue;
                    if constexpr (NEW) plane_n[ob + pe_m[m]] = xn[m];
                    if constexpr (OLD) part[ob + pe_m[m]] = wk * un[m];
                }
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    xr[m] = xn[m];
                    if constexpr (OLD) ur[m] = un[m];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                aEn[j][m] = bEn[j][m];
                aQn[j][m] = bQn[j][m];
                aEo[j][m] = bEo[j][m];
                aQo[j][m] = bQo[j][m];
            }
        }
    }
    if constexpr (NEW) {
        __syncthreads();   // the plane's stores by every lane before the reads below
        // periodic memory of plane kn (I in FP64; the difference form adds S): on the
        // outgoing face along e one vertex per column (plane normal to e, index
        // fz N_d + flipped d = fz N_d + c), and on the last column every vertex (plane
        // normal to d, index fz N_e + flipped e)
        const int par1 = A.parity[f] ^ 1;
        const int64_t rb = ((int64_t)f * A.na + C.ray) * 2 + par1;
        const int fz = A.n[2] - 1 - C.kn;             // rays going down: z flipped
        if (A.periodic[C.e]) {
            double *we = A.wrap[C.e] + rb * ((int64_t)C.Nd * A.n[2]) + (int64_t)fz * C.Nd;
            const int pe_out = C.se > 0 ? C.Ne - 1 : 0;
            for (int c = lane; c < C.Nd; c += 64) {
                const int pd = C.sd > 0 ? c : C.Nd - 1 - c;
                double I = double(plane_n[(int64_t)pd * C.Ne + pe_out]);
                if constexpr (DFORM) I += ghS[pd];
                we[c] = I;
            }
        }
        if (A.periodic[C.d]) {
            double *wd = A.wrap[C.d] + rb * ((int64_t)C.Ne * A.n[2]) + (int64_t)fz * C.Ne;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (!ok_m[m]) continue;
                const int fe = C.se > 0 ? pe_m[m] : C.Ne - 1 - pe_m[m];
                double I = double(xr[m]);
                if constexpr (DFORM) I += ghS[A.nmax + pe_m[m]];
                wd[fe] = I;
            }
        }
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
    __shared__ unsigned char xchain[kGsMaxDown];   // ray di runs as a chain along x
    const int f = blockIdx.y;
    if (A.frozen[f]) return;
    for (int di = threadIdx.x; di < A.nd; di += 256) xchain[di] = A.rays[A.down[di]].d == 0;
    __syncthreads();
    const int nx = A.n[0], ny = A.n[1];
    const int64_t stride_up = (int64_t)A.nf * A.cells;
    unsigned long long rb = 0ull;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < A.pxy) {
        const int x = (int)(p % nx), y = (int)(p / nx);
        const int64_t i = (int64_t)f * A.cells + (int64_t)k * A.pxy + p;
        const int64_t px = (int64_t)x * ny + y;   // chains along x keep the plane y fastest
        const Real *pp = A.part + (int64_t)f * A.pxy;
        const int64_t pstride = (int64_t)A.nf * A.pxy;
        double sum = 0.0;
#pragma unroll
        for (int o = 0; o < 4; ++o) sum += (double)A.part_up[o * stride_up + i];
#pragma unroll 8
        for (int di = 0; di < A.nd; ++di) sum += (double)pp[di * pstride + (xchain[di] ? px : p)];
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
        A.S_t[(int64_t)f * A.cells + (int64_t)k * A.pxy + px] = Sn;
        const double r = (Sn != 0.0) ? fabs(dS) / fabs(Sn) : 0.0;
        rb = (unsigned long long)__double_as_longlong(r);
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

// [nf][nz][ny][nx] -> [nf][nz][nx][ny] through a 32 x 32 LDS tile (coalesced on both
// sides); blockIdx.z runs over the bins and planes.
template <typename T>
__global__ void __launch_bounds__(256) gs_transpose_kernel(const T *src, T *dst, int nx, int ny)
{
    __shared__ T tile[32][33];
    const int64_t base = (int64_t)blockIdx.z * nx * ny;
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int x = x0 + tx, y = y0 + j;
        if (x < nx && y < ny) tile[j][tx] = src[base + (int64_t)y * nx + x];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int y = y0 + tx, x = x0 + j;
        if (x < nx && y < ny) dst[base + (int64_t)x * ny + y] = tile[tx][j];
    }
}

__global__ void gs_clear_kernel(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// e0/e1 (or null): events that take the start and end time of this dispatch
template <typename Real, bool DF, int M, bool NEW, bool OLD, bool FULL>
void launch_chain_k(const GsArgs<Real> &A, int t, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid((unsigned)A.ns, (unsigned)A.nf);
    if (e0 || e1)
        hipExtLaunchKernelGGL(gs_chain_kernel<Real, DF, M, NEW, OLD, FULL>, grid, dim3(64), 0, st, e0, e1, 0, A, t);
    else
        hipLaunchKernelGGL((gs_chain_kernel<Real, DF, M, NEW, OLD, FULL>), grid, dim3(64), 0, st, A, t);
}

template <typename Real, bool DF, int M, bool FULL>
void launch_chain_f(const GsArgs<Real> &A, int t, int kind, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    if (kind == 0)
        launch_chain_k<Real, DF, M, false, true, FULL>(A, t, st, e0, e1);
    else if (kind == 1)
        launch_chain_k<Real, DF, M, true, true, FULL>(A, t, st, e0, e1);
    else
        launch_chain_k<Real, DF, M, true, false, FULL>(A, t, st, e0, e1);
}

template <typename Real, bool DF, int M>
void launch_chain_m(const GsArgs<Real> &A, int t, int kind, bool full, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    if (full)
        launch_chain_f<Real, DF, M, true>(A, t, kind, st, e0, e1);
    else
        launch_chain_f<Real, DF, M, false>(A, t, kind, st, e0, e1);
}

}  // namespace

template <typename Real>
hipError_t launch_gs_plane(const GsArgs<Real> &A, int t, hipStream_t st, hipEvent_t before, hipEvent_t after)
{
    constexpr bool DF = sizeof(Real) == 4;
    const int64_t cb = (A.pxy + 255) / 256;
    const int64_t coef_blocks = A.ns > 0 ? 8 * ((A.ns + 7) / 8) * cb : 0;
    const int64_t blocks = A.steep_blocks + coef_blocks;
    if (blocks > 0)
        hipLaunchKernelGGL((gs_prep_kernel<Real, DF>), dim3((unsigned)blocks, (unsigned)A.nf), dim3(256), 0, st, A, t);
    if (A.ns > 0) {
        const int ne = std::max(A.n[0], A.n[1]);
        const int M = ne <= 64 ? 1 : (ne <= 128 ? 2 : 4);
        // every chain's lanes are full when both in-plane extents are 64 M
        const bool full = A.n[0] == 64 * M && A.n[1] == 64 * M;
        const int nz = A.n[2];
        const int kind = t == 0 ? 0 : (t == nz ? 2 : 1);   // old only, both, new only
        if (M == 1)
            launch_chain_m<Real, DF, 1>(A, t, kind, full, st, before, after);
        else if (M == 2)
            launch_chain_m<Real, DF, 2>(A, t, kind, full, st, before, after);
        else
            launch_chain_m<Real, DF, 4>(A, t, kind, full, st, before, after);
    }
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_gs_update(const GsArgs<Real> &A, int k, hipStream_t st)
{
    constexpr bool DF = sizeof(Real) == 4;
    hipLaunchKernelGGL((gs_update_kernel<Real, DF>), dim3((unsigned)((A.pxy + 255) / 256), (unsigned)A.nf), dim3(256),
                       0, st, A, k);
    return hipGetLastError();
}

hipError_t launch_gs_clear(unsigned long long *blockmax, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(gs_clear_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, blockmax, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_transpose(const T *src, T *dst, int nf, const int n[3], hipStream_t st)
{
    hipLaunchKernelGGL((gs_transpose_kernel<T>), dim3((unsigned)((n[0] + 31) / 32), (unsigned)((n[1] + 31) / 32),
                                                     (unsigned)((int64_t)nf * n[2])),
                       dim3(256), 0, st, src, dst, n[0], n[1]);
    return hipGetLastError();
}

template hipError_t launch_gs_transpose<float>(const float *, float *, int, const int[3], hipStream_t);
template hipError_t launch_gs_transpose<double>(const double *, double *, int, const int[3], hipStream_t);
template hipError_t launch_gs_plane<float>(const GsArgs<float> &, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_gs_plane<double>(const GsArgs<double> &, int, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_gs_update<float>(const GsArgs<float> &, int, hipStream_t);
template hipError_t launch_gs_update<double>(const GsArgs<double> &, int, hipStream_t);

}  // namespace rtsc
