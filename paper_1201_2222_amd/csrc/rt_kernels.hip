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
// previous plane, so the lanes of the wave update a whole T x T plane at once.
// chi and S of the tile plus its upwind halo are staged in LDS once and shared by
// all rays of the octant; before its plane loop a wave loads every upwind-halo
// intensity the ray will need (the neighbour tiles' downwind faces, periodic
// memory or boundary values) into LDS in one batch, so the plane loop itself
// touches only LDS.
#include <hip/hip_runtime.h>

#include "rt_internal.h"
#include "rt_device.h"

namespace rtsc {

namespace {

constexpr int T = kTile;
constexpr int TP = T + 1;            // tile plus one upwind halo layer
// LDS cubes are stored with row pitch CUBE_P and plane pitch CUBE_Q (x fastest):
// with the lanes of a wave on an 8 x 8 plane, pitches 9 and 88 give no LDS bank
// conflicts for rays crossing x or y planes first and two-way conflicts for z (a
// dense 9^3 cube has two-way conflicts on all three).
constexpr int CUBE_P = 9, CUBE_Q = 88;
constexpr int TILE_LDS = (TP - 1) * (1 + CUBE_P + CUBE_Q) + 1;   // words of a cube
// chi and S are staged with the upwind halo, and for the second-order form also the
// downwind layer (the downwind point of each vertex lies in the next plane):
// edge TP, or TP + 1 with ORD = 1.
template <int ORD>
constexpr int stage_edge() { return ORD ? TP + 1 : TP; }
template <int ORD>
constexpr int stage_p() { return ORD ? 11 : CUBE_P; }      // pitches of the staged cube (edge 10: 11, 120)
template <int ORD>
constexpr int stage_q() { return ORD ? 120 : CUBE_Q; }
template <int ORD>
constexpr int stage_cells() { return (stage_edge<ORD>() - 1) * (1 + stage_p<ORD>() + stage_q<ORD>()) + 1; }
// Reals of LDS per wave: the cube of I (or D) of its current ray, and when a wave
// sweeps several rays of a tile (multi) nq partial-sum tiles that accumulate them
constexpr int wave_lds(int nq, bool multi) { return TILE_LDS + (multi ? nq * T * T * T : 0); }
constexpr int NMOM = 10;             // moments mode: J, H_x,y,z, K_xx,yy,zz,xy,xz,yz

// Workgroup barrier for LDS traffic only: no wait for outstanding global stores
// (__syncthreads also orders global memory, which makes it wait for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Order of one wave's LDS accesses across lanes.  The LDS executes a wave's
// operations in issue order, so a store followed by loads of other lanes' words
// needs no wait; this only keeps the compiler from moving LDS accesses across.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wave_lds_sync()
{
    // make this wave's LDS stores visible to its other lanes (lgkmcnt(0)) and keep
    // the compiler from moving LDS accesses across this point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave's global stores have completed (vmcnt(0): the memory system has taken
// them) before the workgroup barrier that precedes the publication of its tile.
__device__ __forceinline__ void tile_stores_done()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt and lgkmcnt not waited for
}

// ---- second-order segment (section 3.3, eq. rtdisc with Bezier source) -------------
// Over an upwind segment of optical depth x the source is the quadratic Bezier curve
// from S0 (u = 0) through the control point Sc to S- (u = 1), u = t/x, and
//   I0 = I- E + alpha S- + beta S0 + gamma Sc,
//   alpha = int_0^x u^2 e^-t, gamma = int 2u(1-u) e^-t, beta = int (1-u)^2 e^-t.
// With e1 = 1 - E(1 + x), e2 = 2 - E(x^2 + 2x + 2):  alpha = e2/x^2,
// gamma = 2 e1/x - 2 e2/x^2, beta = (1 - E) - alpha - gamma.  For small x these
// cancel; there all three follow from the one series F3(x) = sum_n (-x)^n/(n+3)!:
//   beta = 2x F3,  gamma = x (1 - 2(x + 2) F3),  alpha = x ((x^2 + 2x + 2) F3 - x/2)
// (substitute (1 - E) = x - x^2/2 + x^3 F3 into the closed forms).  One series keeps
// the number of distinct constants, which the compiler holds in scalar registers
// across the sweep, small.
// 1/(n+3)!, n = 0 .. 15
#define RT_INV_FACT3                                                                                         \
    {1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0, 1.0 / 40320.0, 1.0 / 362880.0,          \
     1.0 / 3628800.0, 1.0 / 39916800.0, 1.0 / 479001600.0, 1.0 / 6227020800.0, 1.0 / 87178291200.0,        \
     1.0 / 1307674368000.0, 1.0 / 20922789888000.0, 1.0 / 355687428096000.0, 1.0 / 6402373705728000.0}

// FP64 (plain form and Lambda*): series below x = 0.5 (16 terms).
__device__ __forceinline__ void bezier_coeffs(double x, double &E, double &al, double &be, double &ga)
{
    E = exp(-x);
    if (x < 0.5) {
        constexpr int N = 16;
        const double c[N] = RT_INV_FACT3;
        double f = c[N - 1];
#pragma unroll
        for (int n = N - 2; n >= 0; --n) f = c[n] - x * f;
        be = 2.0 * x * f;
        ga = x * (1.0 - 2.0 * (x + 2.0) * f);
        al = x * (((x + 2.0) * x + 2.0) * f - 0.5 * x);
    } else {
        const double e0 = -expm1(-x);
        const double e1 = 1.0 - E * (1.0 + x);
        const double e2 = 2.0 - E * (x * x + 2.0 * x + 2.0);
        al = e2 / (x * x);
        ga = 2.0 * e1 / x - 2.0 * e2 / (x * x);
        be = e0 - al - ga;
    }
}

// FP32, difference form: with E + alpha + beta + gamma = 1 the plain form becomes
//   D0 = D- E + (E + alpha)(S- - S0) + gamma (Sc - S0),
// so only E, E + alpha and gamma are needed.  Series below x = 1 (10 terms); both
// branches are evaluated and one selected.
__device__ __forceinline__ void bezier_coeffs(float x, float &E, float &Ea, float &ga)
{
    E = __expf(-x);
    constexpr int N = 10;
    const double c[16] = RT_INV_FACT3;
    const float m = -x;
    float f = float(c[N - 1]);
#pragma unroll
    for (int n = N - 2; n >= 0; --n) f = fmaf(m, f, float(c[n]));
    const float as = x * (((x + 2.0f) * x + 2.0f) * f - 0.5f * x);
    const float gs = x * (1.0f - 2.0f * (x + 2.0f) * f);
    const float r = __builtin_amdgcn_rcpf(x);
    const float e1 = 1.0f - E * (1.0f + x);
    const float e2 = 2.0f - E * ((x + 2.0f) * x + 2.0f);
    const float ac = e2 * r * r;
    const float gc = 2.0f * e1 * r - 2.0f * ac;
    const bool small = x < 1.0f;
    Ea = E + (small ? as : ac);
    ga = small ? gs : gc;
}

// Control point relative to S0 (section 3.3): Sc - S0 = -(h1/2) S' with S' the slope
// at the vertex of the parabola through (-h1, S-), (0, S0), (h2, S+) in optical depth.
// With a = S- - S0, b = S+ - S0 and t = h1/h2 this is (a - b t^2) / (2 (1 + t)); with
// h2 = 0 the one-sided slope gives a/2 (and h1 = 0 leaves the segment without
// weight).  The result is clamped to lie between S- and S0, i.e. between a and 0.
// t is capped where t^2 would overflow; there the value is clamped anyway, and for
// b = 0 it stays ~0 as it should.
__device__ __forceinline__ float fdiv(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double fdiv(double n, double d) { return n / d; }

template <typename Real>
__device__ __forceinline__ Real control_offset(Real a, Real b, Real h1, Real h2)
{
    constexpr Real tmax = sizeof(Real) == 4 ? Real(1e18) : Real(1e150);
    const bool one_sided = !(h2 > Real(0));
    Real t = fdiv(h1, one_sided ? Real(1) : h2);
    t = t < tmax ? t : tmax;
    Real dc = fdiv(a - b * t * t, Real(2) * (Real(1) + t));
    dc = one_sided ? Real(0.5) * a : dc;
    const Real lo = a < Real(0) ? a : Real(0), hi = a < Real(0) ? Real(0) : a;
    dc = dc < lo ? lo : dc;
    dc = dc > hi ? hi : dc;
    return dc;
}

// Per-workgroup tile description, all scalars (no arrays indexed by a runtime axis).
struct TileCtx {
    int f, par;
    int sgx, sgy, sgz;
    int tx, ty, tz;
    int g0x, g0y, g0z;
    int ex, ey, ez;
    int64_t fbase;   // f * cells
};

// Where the value of one ray at a ghost vertex (vx, vy, vz) in flipped coordinates
// (a coordinate of -1) comes from: *src (nullptr: zero incident intensity), and in
// the difference form minus S at *scell.  chi and S of a ghost are those of the
// folded vertex.
template <typename Real>
__device__ __forceinline__ void ghost_source(const SweepArgs<Real> &A, const TileCtx &c, int vx, int vy, int vz,
                                             int ray, int gidx, const double *&src, int64_t &scell)
{
    const bool ox = vx < 0, oy = vy < 0, oz = vz < 0;
    const int64_t rb = (int64_t)c.f * A.na + ray;
    const int rx = fold(to_real(vx, c.sgx, A.n[0]), A.n[0], A.periodic[0]);
    const int ry = fold(to_real(vy, c.sgy, A.n[1]), A.n[1], A.periodic[1]);
    const int rz = fold(to_real(vz, c.sgz, A.n[2]), A.n[2], A.periodic[2]);
    scell = c.fbase + ((int64_t)rz * A.n[1] + ry) * A.n[0] + rx;
    // outside a non-periodic face: that face's condition, z before y before x
    int q = -1;
    if (oz && !A.periodic[2]) q = 2;
    else if (oy && !A.periodic[1]) q = 1;
    else if (ox && !A.periodic[0]) q = 0;
    if (q >= 0) {
        const int lo = sel3(q, c.sgx, c.sgy, c.sgz) > 0;
        const int kind = lo ? sel3(q, A.bc_lo[0], A.bc_lo[1], A.bc_lo[2]) : sel3(q, A.bc_hi[0], A.bc_hi[1], A.bc_hi[2]);
        src = nullptr;
        if (kind == BC_THERMAL) {
            src = A.B + scell;
        } else if (kind == BC_FIXED) {
            const double *F = (q == 0) ? (lo ? A.fixed[0] : A.fixed[1])
                                       : (q == 1 ? (lo ? A.fixed[2] : A.fixed[3]) : (lo ? A.fixed[4] : A.fixed[5]));
            const int64_t pidx = (q == 0) ? (int64_t)rz * A.n[1] + ry
                                          : (q == 1 ? (int64_t)rz * A.n[0] + rx : (int64_t)ry * A.n[0] + rx);
            const int64_t P = sel3(q, A.plane[0], A.plane[1], A.plane[2]);
            src = F + ((int64_t)c.f * A.na + gidx) * P + pidx;
        }
        return;
    }
    // only periodic axes are outside: the previous sweep's intensity at the
    // wrapped vertex, kept on the ray's outgoing plane
    const int wx = ox ? A.n[0] - 1 : vx, wy = oy ? A.n[1] - 1 : vy, wz = oz ? A.n[2] - 1 : vz;
    if (ox)
        src = A.wrap[0] + (rb * 2 + c.par) * A.plane[0] + (int64_t)wz * A.n[1] + wy;
    else if (oy)
        src = A.wrap[1] + (rb * 2 + c.par) * A.plane[1] + (int64_t)wz * A.n[0] + wx;
    else
        src = A.wrap[2] + (rb * 2 + c.par) * A.plane[2] + (int64_t)wy * A.n[0] + wx;
}

// The upwind shell of one ray's LDS cube: the planes x = -1, y = -1 and z = -1 of
// the tile in flipped local coordinates, edges and corner included (the cube has
// the staged tile's layout), 217 vertices.  Each comes from the padded face plane of
// its axis at the tile's slot: the downwind face of the upwind neighbour tile, or a
// ghost value written before the sweep.  Lane l loads vertex (u, w) = (l & 7, l >> 3)
// of the interior (8 x 8) of each of the three planes, and lanes 0 .. 24 one of the 25
// vertices on the cube's edges at -1: x plane row z = -1 (9, corner included), x plane
// column y = -1 (8), y plane row z = -1 (8).  Offsets inside a slot are 32-bit and
// the slot bases wave-uniform.  shell_load issues the loads into registers and
// shell_store writes them into the cube, so the loads of the next ray are in flight
// while a ray is swept.
constexpr int SHELL_PER_LANE = 4;

template <typename Real>
struct Shell {
    Real v[SHELL_PER_LANE];
    int slot[SHELL_PER_LANE];    // cube index, -1: none
};

template <typename Real>
__device__ __forceinline__ void shell_load(const SweepArgs<Real> &A, const TileCtx &c, int ray, int lane, Shell<Real> &sh)
{
    const int64_t rb = (int64_t)c.f * A.na + ray;
    const Real *bx = A.face[0] + (rb * A.nt[0] + c.tx) * A.pplane[0];
    const Real *by = A.face[1] + (rb * A.nt[1] + c.ty) * A.pplane[1];
    const Real *bz = A.face[2] + (rb * A.nt[2] + c.tz) * A.pplane[2];
    const FacePlane Fx(A.n[1], A.n[2]), Fy(A.n[0], A.n[2]), Fz(A.n[0], A.n[1]);
    const int u = lane & (T - 1), w = lane / T;
    // interiors: x plane (y, z) = (u, w); y plane (x, z) = (u, w); z plane (x, y) = (u, w);
    // each one aligned 8 x 8 block
    const bool okx = u < c.ey && w < c.ez, oky = u < c.ex && w < c.ez, okz = u < c.ex && w < c.ey;
    const uint32_t ox = (uint32_t)(Fx.blk(c.ty, c.tz) + lane);   // lane = 8 w + u
    const uint32_t oy = (uint32_t)(Fy.blk(c.tx, c.tz) + lane);
    const uint32_t oz = (uint32_t)(Fz.blk(c.tx, c.ty) + lane);
    sh.slot[0] = okx ? (w + 1) * CUBE_Q + (u + 1) * CUBE_P : -1;
    sh.slot[1] = oky ? (w + 1) * CUBE_Q + (u + 1) : -1;
    sh.slot[2] = okz ? (w + 1) * CUBE_P + (u + 1) : -1;
    sh.v[0] = okx ? bx[ox] : Real(0);
    sh.v[1] = oky ? by[oy] : Real(0);
    sh.v[2] = okz ? bz[oz] : Real(0);
    // edges
    const int e = lane;
    const bool row_x = e < TP, col_x = e >= TP && e < TP + T, row_y = e >= TP + T && e < TP + 2 * T;
    const int j = row_x ? e : (col_x ? e - TP : e - TP - T);   // position along the edge
    bool oke;
    uint32_t oe;
    int se;
    if (row_x) {            // x plane, z = -1, y = j - 1: the last row of the block below
        oke = j <= c.ey;
        oe = (uint32_t)Fx.at(c.g0y + j - 1, c.g0z - 1);
        se = j * CUBE_P;
    } else if (col_x) {     // x plane, y = -1, z = j: the copied last column of the block beside
        oke = j < c.ez;
        oe = (uint32_t)(c.ty > 0 ? Fx.colblk(c.ty - 1, c.tz) + j : Fx.at(-1, c.g0z + j));
        se = (j + 1) * CUBE_Q;
    } else {                // y plane, z = -1, x = j
        oke = row_y && j < c.ex;
        oe = (uint32_t)Fy.at(c.g0x + j, c.g0z - 1);
        se = j + 1;
    }
    sh.slot[3] = oke ? se : -1;
    sh.v[3] = oke ? (row_y ? by : bx)[oe] : Real(0);
}

template <typename Real>
__device__ __forceinline__ void shell_store(const Shell<Real> &sh, Real *Ic)
{
#pragma unroll
    for (int k = 0; k < SHELL_PER_LANE; ++k)
        if (sh.slot[k] >= 0) Ic[sh.slot[k]] = sh.v[k];
}

// The downwind faces of the tile for one ray, read from its cube after the sweep:
// interior faces go to the next tile's slot of the padded face planes; the grid's
// last faces on periodic axes feed the next sweep's periodic memory (which keeps I,
// in FP64).
template <typename Real, bool DFORM, int ORD>
__device__ void write_faces(const SweepArgs<Real> &A, const TileCtx &c, int ray, int lane, const Real *Ic,
                            const double *SL)
{
    constexpr int SP = stage_p<ORD>(), SQ = stage_q<ORD>();   // pitches of the staged S cube
    const int64_t rb = (int64_t)c.f * A.na + ray;
    const int u = lane % T, w = lane / T;   // T * T == 64 face vertices, one per lane
    // Per axis q the face goes to the next tile's slot of the padded planes (interior)
    // or, behind the grid's last tile on a periodic axis, to the periodic memory; the
    // choice is wave-uniform.  Bases are wave-uniform, offsets 32-bit.  Every value
    // first, then the stores back to back (a register that a store still reads must
    // not be reused before the store has completed).
    const bool inx = c.tx < A.nt[0] - 1, iny = c.ty < A.nt[1] - 1, inz = c.tz < A.nt[2] - 1;
    Real *fx = A.face[0] + (rb * A.nt[0] + c.tx + 1) * A.pplane[0];
    Real *fy = A.face[1] + (rb * A.nt[1] + c.ty + 1) * A.pplane[1];
    Real *fz = A.face[2] + (rb * A.nt[2] + c.tz + 1) * A.pplane[2];
    double *wx = A.wrap[0] + (rb * 2 + (c.par ^ 1)) * A.plane[0];
    double *wy = A.wrap[1] + (rb * 2 + (c.par ^ 1)) * A.plane[1];
    double *wz = A.wrap[2] + (rb * 2 + (c.par ^ 1)) * A.plane[2];
    const bool px = !inx && A.periodic[0], py = !iny && A.periodic[1], pz = !inz && A.periodic[2];
    // x face: (y, z) = (u, w); y face: (x, z) = (u, w); z face: (x, y) = (u, w)
    const bool okx = u < c.ey && w < c.ez, oky = u < c.ex && w < c.ez, okz = u < c.ex && w < c.ey;
    const Real vx = Ic[(w + 1) * CUBE_Q + (u + 1) * CUBE_P + c.ex];
    const Real vy = Ic[(w + 1) * CUBE_Q + c.ey * CUBE_P + (u + 1)];
    const Real vz = Ic[c.ez * CUBE_Q + (w + 1) * CUBE_P + (u + 1)];
    double ix = double(vx), iy = double(vy), iz = double(vz);
    if constexpr (DFORM) {   // the periodic memory keeps I = D + S
        ix += SL[(w + 1) * SQ + (u + 1) * SP + c.ex];
        iy += SL[(w + 1) * SQ + c.ey * SP + (u + 1)];
        iz += SL[c.ez * SQ + (w + 1) * SP + (u + 1)];
    }
    const FacePlane Fx(A.n[1], A.n[2]), Fy(A.n[0], A.n[2]), Fz(A.n[0], A.n[1]);
    const uint32_t ofx = (uint32_t)(Fx.blk(c.ty, c.tz) + lane);   // lane = 8 w + u
    const uint32_t ofy = (uint32_t)(Fy.blk(c.tx, c.tz) + lane);
    const uint32_t ofz = (uint32_t)(Fz.blk(c.tx, c.ty) + lane);
    // lanes on a full block's last column also write its copy (read by the next tile
    // along a as its halo column)
    const bool lastc = u == T - 1;
    const uint32_t cfx = (uint32_t)(Fx.colblk(c.ty, c.tz) + w);
    const uint32_t cfy = (uint32_t)(Fy.colblk(c.tx, c.tz) + w);
    const uint32_t cfz = (uint32_t)(Fz.colblk(c.tx, c.ty) + w);
    const uint32_t owx = (uint32_t)((c.g0z + w) * A.n[1] + (c.g0y + u));
    const uint32_t owy = (uint32_t)((c.g0z + w) * A.n[0] + (c.g0x + u));
    const uint32_t owz = (uint32_t)((c.g0y + w) * A.n[0] + (c.g0x + u));
    if (okx) {
        if (inx) {
            fx[ofx] = vx;
            if (lastc) fx[cfx] = vx;
        } else if (px) {
            wx[owx] = ix;
        }
    }
    if (oky) {
        if (iny) {
            fy[ofy] = vy;
            if (lastc) fy[cfy] = vy;
        } else if (py) {
            wy[owy] = iy;
        }
    }
    if (okz) {
        if (inz) {
            fz[ofz] = vz;
            if (lastc) fz[cfz] = vz;
        } else if (pz) {
            wz[owz] = iz;
        }
    }
}

constexpr int lds_stride(int q) { return q == 0 ? 1 : (q == 1 ? CUBE_P : CUBE_Q); }
template <int ORD>
constexpr int stage_stride(int q) { return q == 0 ? 1 : (q == 1 ? stage_p<ORD>() : stage_q<ORD>()); }
constexpr int tile_stride(int q) { return q == 0 ? 1 : (q == 1 ? T : T * T); }

// Plane-by-plane sweep of one ray through the tile along its first-crossed axis D
// (all strides compile-time).  Lane (ia, ib) owns one vertex of every plane.
// Weight of a ray in accumulated quantity q: w (J); moments mode also w mu_i (H)
// and w mu_i mu_j (K, order xx yy zz xy xz yz).  Products formed as in the sweep.
template <typename Real, int NQ>
__device__ __forceinline__ Real ray_weight(const RayGeo *G, int q)
{
    const double wd = G->wk;
    if (NQ == 1 || q == 0) return Real(wd);
    const double mx = G->mu[0], my = G->mu[1], mz = G->mu[2];
    switch (q) {
    case 1: return Real(wd * mx);
    case 2: return Real(wd * my);
    case 3: return Real(wd * mz);
    case 4: return Real(wd * mx * mx);
    case 5: return Real(wd * my * my);
    case 6: return Real(wd * mz * mz);
    case 7: return Real(wd * mx * my);
    case 8: return Real(wd * mx * mz);
    default: return Real(wd * my * mz);
    }
}

// Upwind and own chi and S of one vertex of a plane, as loaded from the staged tile,
// and for the second-order form the downwind chi (p..) and S (t..).
template <typename Real>
struct SegIn {
    Real c00, c10, c01, c11, c0;
    double s00, s10, s01, s11, s0;
    Real p00, p10, p01, p11;
    double t00, t10, t01, t11;
};

// ORD = 0: first order (linear source between S- and S0).  ORD = 1: second order
// (quadratic Bezier source with the control point from S-, S0 and the downwind S+).
template <typename Real, bool ACC, int NQ, int D, bool DFORM, int ORD>
__device__ __forceinline__ void ray_planes(const RayGeo *G, int lane, Real *Ic,
                                           const Real *chiL, const double *SL, Real *Jw)
{
    constexpr int DA = (D == 0) ? 1 : 0, DB = (D == 2) ? 1 : 2;
    constexpr int SD = lds_stride(D), SA = lds_stride(DA), SB = lds_stride(DB);
    constexpr int XD = stage_stride<ORD>(D), XA = stage_stride<ORD>(DA), XB = stage_stride<ORD>(DB);
    constexpr int JD = tile_stride(D), JA = tile_stride(DA), JB = tile_stride(DB);
    const int ia = lane & (T - 1), ib = lane / T;
    const int lb = (ia + 1) * SA + (ib + 1) * SB;    // in the cube of I
    const int ls = (ia + 1) * XA + (ib + 1) * XB;    // in the staged chi and S
    const int jbase = ia * JA + ib * JB;
    const Real s_half = Real(0.5 * G->s);
    const Real w00 = Real(G->w4[0]), w10 = Real(G->w4[1]), w01 = Real(G->w4[2]), w11 = Real(G->w4[3]);
    const double w00d = G->w4[0], w10d = G->w4[1], w01d = G->w4[2], w11d = G->w4[3];
    // weights of this ray in the accumulated quantities: w (J), and in moments mode
    // also w mu_i (H) and w mu_i mu_j (K)
    Real cq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) cq[q] = ray_weight<Real, NQ>(G, q);
    // Per plane, v = I- E + c with the attenuation E and the source term c of the
    // segment; they do not depend on the intensity, so their loads run two planes
    // ahead and their arithmetic one plane ahead of the recurrence.
    auto load_seg = [&](int p) {
        const int l0 = ls + (p + 1) * XD;
        const int lu = l0 - XD;
        SegIn<Real> x;
        x.c00 = chiL[lu];
        x.c10 = chiL[lu - XA];
        x.c01 = chiL[lu - XB];
        x.c11 = chiL[lu - XA - XB];
        x.c0 = chiL[l0];
        x.s00 = SL[lu];
        x.s10 = SL[lu - XA];
        x.s01 = SL[lu - XB];
        x.s11 = SL[lu - XA - XB];
        x.s0 = SL[l0];
        if constexpr (ORD == 1) {
            // the downwind point mirrors the upwind one through the vertex
            const int ld = l0 + XD;
            x.p00 = chiL[ld];
            x.p10 = chiL[ld + XA];
            x.p01 = chiL[ld + XB];
            x.p11 = chiL[ld + XA + XB];
            x.t00 = SL[ld];
            x.t10 = SL[ld + XA];
            x.t01 = SL[ld + XB];
            x.t11 = SL[ld + XA + XB];
        }
        return x;
    };
    auto seg = [&](const SegIn<Real> &x, Real &E, Real &cc) {
        const Real Cm = w00 * x.c00 + w10 * x.c10 + w01 * x.c01 + w11 * x.c11;
        const Real dt = s_half * (Cm + x.c0);
        const double Sm = w00d * x.s00 + w10d * x.s10 + w01d * x.s01 + w11d * x.s11;
        if constexpr (ORD == 1) {
            const Real Cp = w00 * x.p00 + w10 * x.p10 + w01 * x.p01 + w11 * x.p11;
            const Real dtp = s_half * (x.c0 + Cp);   // optical depth of the downwind segment
            const double Sp = w00d * x.t00 + w10d * x.t10 + w01d * x.t01 + w11d * x.t11;
            if constexpr (DFORM) {
                Real Ea, ga;
                bezier_coeffs(dt, E, Ea, ga);
                const Real a = Real(Sm - x.s0), b = Real(Sp - x.s0);   // differences formed in FP64
                cc = Ea * a + ga * control_offset<Real>(a, b, dt, dtp);
            } else {
                double al, be, ga;
                bezier_coeffs(dt, E, al, be, ga);
                const double Sc = x.s0 + control_offset<double>(Sm - x.s0, Sp - x.s0, dt, dtp);
                cc = (al * Sm + be * x.s0) + ga * Sc;
            }
        } else if constexpr (DFORM) {
            Real g;
            seg_coeffs(dt, E, g);
            cc = Real(Sm - x.s0) * g;   // S- - S0 formed in FP64
        } else {
            Real pm, p0;
            seg_coeffs(dt, E, pm, p0);
            cc = pm * Real(Sm) + p0 * Real(x.s0);
        }
    };
    // The recurrence along the ray, one plane per step.  Every lane steps every plane
    // (no branch, so the loads running ahead need no register copies at a join): a
    // lane outside a ragged tile, and a plane past its end, write only cube entries no
    // active lane reads.
    // When the wave sweeps several rays of the tile (ACC), w v (and in moments mode
    // w mu v, w mu mu v) is added to its partial-sum tiles per vertex; with one ray
    // per wave the cube itself keeps v for the sum over the waves.
    Real E, cc;
    seg(load_seg(0), E, cc);
    SegIn<Real> nx = load_seg(1);
#pragma unroll
    for (int p = 0; p < T; ++p) {
        {
            const int l0 = lb + (p + 1) * SD;
            const int lu = l0 - SD;
            const Real i00 = Ic[lu], i10 = Ic[lu - SA], i01 = Ic[lu - SB], i11 = Ic[lu - SA - SB];
            SegIn<Real> nn;
            if (p + 2 < T) nn = load_seg(p + 2);   // inside the cube even past a ragged edge
            Real En = Real(0), ccn = Real(0);
            if (p + 1 < T) seg(nx, En, ccn);
            const Real v = (w00 * i00 + w10 * i10 + w01 * i01 + w11 * i11) * E + cc;
            Ic[l0] = v;
            if constexpr (ACC) {
                // every lane adds (a lane outside a ragged tile adds to an entry the sum
                // over the waves never reads), so the read of the entry needs no branch
                // and goes out with the plane's other loads
                const int j = jbase + p * JD;
#pragma unroll
                for (int q = 0; q < NQ; ++q) Jw[q * T * T * T + j] += cq[q] * v;
            }
            wave_lds_order();
            E = En;
            cc = ccn;
            if (p + 2 < T) nx = nn;
        }
    }
}

// Wait until a tile's completion flag carries this sweep's epoch.  The loop polls
// with relaxed agent-scope loads (no cache invalidation per poll); the caller takes
// one agent-scope acquire fence after all of a tile's waits.  The wait is bounded by
// the constant-rate wall clock (limit_ticks) and gives up at once when another wait
// has already run out (*err set), so every wave exits.
__device__ __forceinline__ bool wait_done(const int *flag, int epoch, const int *err, uint64_t limit_ticks)
{
    const uint64_t t0 = wall_clock64();
    for (int i = 0;; ++i) {
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) return true;
        if ((i & 15) == 15) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
            if (wall_clock64() - t0 > limit_ticks) return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// A wave's ray geometry goes through LDS: lanes 0 .. GEO_WORDS - 1 load one word
// each (issued with the other loads of the tile), then store it in the wave's slot.
constexpr int GEO_BYTES = 128;
constexpr int GEO_WORDS = sizeof(RayGeo) / 4;
static_assert(sizeof(RayGeo) <= GEO_BYTES && sizeof(RayGeo) % 4 == 0, "ray geometry slot");

template <typename Real>
__device__ __forceinline__ uint32_t geo_load(const SweepArgs<Real> &A, int ray, bool valid, int lane)
{
    return (valid && lane < GEO_WORDS) ? reinterpret_cast<const uint32_t *>(A.rays + ray)[lane] : 0u;
}

// One tile of one octant and bin: stage chi and S with the upwind halo, sweep every
// ray of the octant through it, write the octant's partial sums.  In the persistent
// sweep (PERSIST) the upwind face-neighbour tiles are awaited after the staging loads
// have been issued and before any face data is read.
template <typename Real, bool DFORM, bool PERSIST, int NQ, bool MULTI, int ORD>
__device__ __forceinline__ void sweep_tile(const SweepArgs<Real> &A, int oct, int f, int packed, int par,
                                           unsigned char *lds_raw, const int *done, int epoch, int ntiles, int nt0,
                                           int nt1, int *err, uint64_t limit_ticks)
{
    const int W = blockDim.x >> 6;
    constexpr int SE = stage_edge<ORD>(), NL = SE * SE * SE, NS = stage_cells<ORD>();
    constexpr int SP = stage_p<ORD>(), SQ = stage_q<ORD>();
    // LDS: per-wave ray geometry, staged S and chi, per-wave cube and partial sums
    uint32_t *geoL = reinterpret_cast<uint32_t *>(lds_raw);
    double *SL = reinterpret_cast<double *>(lds_raw + W * GEO_BYTES);
    Real *chiL = reinterpret_cast<Real *>(SL + NS);
    Real *waveL = chiL + NS;

    TileCtx c;
    c.f = f;
    c.par = par;
    c.fbase = (int64_t)f * A.cells;
    c.sgx = (oct & 1) ? -1 : 1;
    c.sgy = (oct & 2) ? -1 : 1;
    c.sgz = (oct & 4) ? -1 : 1;
    c.tx = packed & 1023;
    c.ty = (packed >> 10) & 1023;
    c.tz = (packed >> 20) & 1023;
    c.g0x = c.tx * T;
    c.g0y = c.ty * T;
    c.g0z = c.tz * T;
    c.ex = min(T, A.n[0] - c.g0x);
    c.ey = min(T, A.n[1] - c.g0y);
    c.ez = min(T, A.n[2] - c.g0z);

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    Real *Ic = waveL + (size_t)wave * wave_lds(NQ, MULTI);   // this wave's cube of I (or D)
    Real *Jw = Ic + TILE_LDS;                                // and its partial-sum tiles (MULTI)
    uint32_t *geo = geoL + wave * (GEO_BYTES / 4);    // and the geometry of its ray
    const RayGeo *G = reinterpret_cast<const RayGeo *>(geo);

    // the first ray's geometry and shell loads go out together with the staging loads
    Shell<Real> sh;
    uint32_t gword = geo_load(A, oct * A.R + wave, wave < A.R, lane);
    if (!PERSIST && wave < A.R) shell_load<Real>(A, c, oct * A.R + wave, lane, sh);

    // ---- stage chi and S of the tile and its upwind halo in LDS --------------------
    // (second order: also the downwind layer).  Each pass issues all of its loads
    // before the first LDS store.  Inside the grid the real cell index is linear in
    // the flipped local coordinates (strides dX, dY, dZ); only tiles whose staged
    // region leaves the grid fold indices per axis.  Indices inside a bin are 32-bit
    // (the library refuses bins of 2^31 or more vertices); lanes without an entry load
    // vertex 0 and store nothing, so the loads need no branch.
    const Real *chif = A.chi + c.fbase;
    const double *Sf = A.S + c.fbase;
    const int dX = c.sgx, dY = c.sgy * A.n[0], dZ = c.sgz * A.n[0] * A.n[1];
    const bool inner = c.tx > 0 && c.ty > 0 && c.tz > 0 &&
                       (ORD == 0 || (c.g0x + T < A.n[0] && c.g0y + T < A.n[1] && c.g0z + T < A.n[2]));
    const int cellH = inner ? (to_real(c.g0z - 1, c.sgz, A.n[2]) * A.n[1] + to_real(c.g0y - 1, c.sgy, A.n[1])) *
                                      A.n[0] + to_real(c.g0x - 1, c.sgx, A.n[0])
                            : 0;
    constexpr int STAGE_K = ORD ? 4 : 3;   // one pass for four or more waves
    for (int base = 0; base < NL; base += STAGE_K * (int)blockDim.x) {
        Real cv[STAGE_K];
        double sv[STAGE_K];
        int li[STAGE_K];
#pragma unroll
        for (int k = 0; k < STAGE_K; ++k) {
            const int idx = base + k * (int)blockDim.x + (int)threadIdx.x;
            const int lx = idx % SE, ly = (idx / SE) % SE, lz = idx / (SE * SE);
            const bool ok = idx < NL && lx <= c.ex + ORD && ly <= c.ey + ORD && lz <= c.ez + ORD;
            int cell;
            if (inner) {
                cell = cellH + (lx * dX + ly * dY + lz * dZ);
            } else {
                const int rx = fold(to_real(c.g0x + lx - 1, c.sgx, A.n[0]), A.n[0], A.periodic[0]);
                const int ry = fold(to_real(c.g0y + ly - 1, c.sgy, A.n[1]), A.n[1], A.periodic[1]);
                const int rz = fold(to_real(c.g0z + lz - 1, c.sgz, A.n[2]), A.n[2], A.periodic[2]);
                cell = (rz * A.n[1] + ry) * A.n[0] + rx;
            }
            const uint32_t uc = ok ? (uint32_t)cell : 0u;
            li[k] = ok ? lx + SP * ly + SQ * lz : -1;
            cv[k] = chif[uc];
            sv[k] = Sf[uc];
        }
#pragma unroll
        for (int k = 0; k < STAGE_K; ++k) {
            if (li[k] < 0) continue;
            chiL[li[k]] = cv[k];
            SL[li[k]] = sv[k];
        }
    }
    if (MULTI)   // several rays per wave accumulate; one ray stores
        for (int k = lane; k < NQ * T * T * T; k += 64) Jw[k] = Real(0);
    if (lane < GEO_WORDS) geo[lane] = gword;
    if (!PERSIST && wave < A.R) shell_store<Real>(sh, Ic);
    if (PERSIST) {
        // upwind face neighbours of this tile in the same octant and bin
        if (threadIdx.x == 0) {
            const int *fl = done + ((int64_t)f * 8 + oct) * ntiles;
            bool ok = true;
            if (c.tx > 0) ok = ok && wait_done(fl + (c.tz * nt1 + c.ty) * nt0 + c.tx - 1, epoch, err, limit_ticks);
            if (c.ty > 0) ok = ok && wait_done(fl + (c.tz * nt1 + c.ty - 1) * nt0 + c.tx, epoch, err, limit_ticks);
            if (c.tz > 0) ok = ok && wait_done(fl + ((c.tz - 1) * nt1 + c.ty) * nt0 + c.tx, epoch, err, limit_ticks);
            // one acquire for the flags read above: the neighbours' faces are visible
            // to this workgroup's loads after the barrier below
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (!ok) atomicOr(err, 1);
        }
        __syncthreads();
        if (wave < A.R) {
            shell_load<Real>(A, c, oct * A.R + wave, lane, sh);
            shell_store<Real>(sh, Ic);
        }
    }
    lds_barrier();

    // ---- per-wave ray sweeps ---------------------------------------------------------
    // The faces of a wave's last ray are written after the partial sums, so no wait
    // for their stores stands between the sweep and the sum.
    int last = -1;
    auto sweep_ray = [&](int ray) {
        const int d = __builtin_amdgcn_readfirstlane(G->d);
        if (d == 0)
            ray_planes<Real, MULTI, NQ, 0, DFORM, ORD>(G, lane, Ic, chiL, SL, Jw);
        else if (d == 1)
            ray_planes<Real, MULTI, NQ, 1, DFORM, ORD>(G, lane, Ic, chiL, SL, Jw);
        else
            ray_planes<Real, MULTI, NQ, 2, DFORM, ORD>(G, lane, Ic, chiL, SL, Jw);
        wave_lds_sync();
    };
    if constexpr (!MULTI) {
        // at most one ray per wave: straight-line code, nothing kept live across rays
        if (wave < A.R) {
            last = oct * A.R + wave;
            sweep_ray(last);
        }
    } else {
        for (int r = wave; r < A.R; r += W) {
            const int ray = oct * A.R + r;
            // the next ray's geometry and shell loads are in flight while this ray is swept
            const bool more = r + W < A.R;
            if (more) {
                gword = geo_load(A, ray + W, true, lane);
                shell_load<Real>(A, c, ray + W, lane, sh);
            }
            sweep_ray(ray);
            if (more) {
                write_faces<Real, DFORM, ORD>(A, c, ray, lane, Ic, SL);
                wave_lds_sync();
                shell_store<Real>(sh, Ic);
                if (lane < GEO_WORDS) geo[lane] = gword;
                wave_lds_sync();
            } else {
                last = ray;
            }
        }
    }
    lds_barrier();

    // ---- fixed-order sum over the waves -> this octant's partial sums --------------
    // layout [8][NQ][nfc][cells], bin f stored at f - f0
    const int64_t cell0 = ((int64_t)to_real(c.g0z, c.sgz, A.n[2]) * A.n[1] + to_real(c.g0y, c.sgy, A.n[1])) * A.n[0] +
                          to_real(c.g0x, c.sgx, A.n[0]);
    // a pass computes all of its sums before its stores (a register a store still
    // reads must not be reused before the store has completed)
    constexpr int COMB_K = 2;
    // Loads of absent waves (w >= W) read wave 0 and are weighted by zero: no
    // branch on W, every load of a vertex goes out at once, and adding the zeros
    // leaves the sum in wave order unchanged.
    Real wkw[kMaxWaves];   // J weights of the waves' rays (one ray per wave), 0 beyond W
#pragma unroll
    for (int w = 0; w < kMaxWaves; ++w) {
        const int wr = w < W ? w : 0;
        wkw[w] = ray_weight<Real, 1>(reinterpret_cast<const RayGeo *>(geoL + wr * (GEO_BYTES / 4)), 0) *
                 Real(w < W ? 1 : 0);
    }
    // this octant's partial sums of bin f, quantity 0, at the tile's first vertex
    Real *pbase = A.part + ((int64_t)oct * NQ * A.nfc + (f - A.f0)) * A.cells + cell0;
    const int64_t qstride = (int64_t)A.nfc * A.cells;
    for (int base = 0; base < NQ * T * T * T; base += COMB_K * (int)blockDim.x) {
        Real acc[COMB_K];
        int64_t off[COMB_K];
        bool ok[COMB_K];
#pragma unroll
        for (int i = 0; i < COMB_K; ++i) {
            const int kq = base + i * (int)blockDim.x + (int)threadIdx.x;
            const int q = kq / (T * T * T), k = kq - q * T * T * T;
            const int lx = k % T, ly = (k / T) % T, lz = k / (T * T);
            ok[i] = kq < NQ * T * T * T && lx < c.ex && ly < c.ey && lz < c.ez;
            off[i] = (NQ == 1 ? 0 : q * qstride) + (lx * dX + ly * dY + lz * dZ);
            acc[i] = Real(0);
            if (!ok[i]) continue;
            // the accumulated tiles (MULTI), or w v from each wave's cube
            Real vw[kMaxWaves];
            const int ci = (lz + 1) * CUBE_Q + (ly + 1) * CUBE_P + (lx + 1);
#pragma unroll
            for (int w = 0; w < kMaxWaves; ++w) {
                const int wr = w < W ? w : 0;
                if constexpr (MULTI) {
                    const Real val = waveL[wr * wave_lds(NQ, true) + TILE_LDS + kq];
                    vw[w] = w < W ? val : Real(0);
                } else {
                    Real cw = wkw[w];
                    if constexpr (NQ != 1)
                        cw = ray_weight<Real, NQ>(reinterpret_cast<const RayGeo *>(geoL + wr * (GEO_BYTES / 4)), q) *
                             Real(w < W ? 1 : 0);
                    vw[w] = cw * waveL[wr * wave_lds(NQ, false) + ci];
                }
            }
            acc[i] = vw[0];
#pragma unroll
            for (int w = 1; w < kMaxWaves; ++w) acc[i] += vw[w];
        }
#pragma unroll
        for (int i = 0; i < COMB_K; ++i)
            if (ok[i]) pbase[off[i]] = acc[i];
    }
    if (last >= 0) write_faces<Real, DFORM, ORD>(A, c, last, lane, Ic, SL);
}

// Waves per SIMD the stage kernel is compiled for.  The FP32 one-ray-per-wave forms
// fit eight (at most 64 VGPRs and 96 SGPRs, no spills), so three workgroups of ten
// waves share a CU; left to itself the compiler settles on 106 SGPRs, seven waves per
// SIMD and two such workgroups.  The other forms keep the compiler's choice.
template <typename Real, bool MULTI>
constexpr int stage_waves_per_simd() { return (sizeof(Real) == 4 && !MULTI) ? 8 : 1; }

// One stage (all tiles with tx + ty + tz = s) of all octants (NOCT = 8) or of the
// octants of the rays going up (NOCT = 4: octants 0 .. 3) and the active bins
// f0 .. f0 + nfc - 1.
template <typename Real, bool DFORM, int NQ, bool MULTI, int ORD, int NOCT = 8>
__global__ void __launch_bounds__(64 * kMaxWaves, (stage_waves_per_simd<Real, MULTI>()))
    sweep_stage_kernel(SweepArgs<Real> A)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int oct = blockIdx.x & (NOCT - 1);
    const int item = blockIdx.x / NOCT;
    const int f = A.f0 + blockIdx.y;
    const int frozen = A.frozen[f];
    const int par = A.parity[f];
    const int packed = A.tiles[A.stage_off + item];
    // the three loads go out together (every value takes part in the test)
    if (frozen | (packed < 0) | (par < 0)) return;
    sweep_tile<Real, DFORM, false, NQ, MULTI, ORD>(A, oct, f, packed, par, lds_raw, nullptr, 0, 0, 0, 0, nullptr, 0);
}

// Batched form: one launch runs stage s of every problem of a batch class (same
// precision and waves per workgroup).  blockIdx.y is the problem; x runs over its
// bins, tiles of stage s and octants.  Problems with fewer stages, and blocks beyond
// a problem's stage, exit at once.
template <typename Real, bool DFORM, bool MULTI, int ORD>
__global__ void __launch_bounds__(64 * kMaxWaves) sweep_batch_stage_kernel(const SweepArgs<Real> *args, int s)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const SweepArgs<Real> &A = args[blockIdx.y];
    if (s >= A.nstages) return;
    const int off = A.stage_tab[s];
    const int per = (A.stage_tab[s + 1] - off) * 8;
    if ((int)blockIdx.x >= per * A.nf) return;
    const int f = (int)blockIdx.x / per;
    const int rem = (int)blockIdx.x - f * per;
    const int oct = rem & 7;
    const int frozen = A.frozen[f];
    const int par = A.parity[f];
    const int packed = A.tiles[off + (rem >> 3)];
    if (frozen | (packed < 0) | (par < 0)) return;
    sweep_tile<Real, DFORM, false, 1, MULTI, ORD>(A, oct, f, packed, par, lds_raw, nullptr, 0, 0, 0, 0, nullptr, 0);
}

// Before each persistent sweep: zero the octants' ticket counters, advance the epoch.
__global__ void dag_begin_kernel(int *counter)
{
    if (threadIdx.x < 8) counter[threadIdx.x] = 0;
    if (threadIdx.x == 0) counter[8] += 1;
}

// Whole formal solution in one launch.  Workgroups with blockIdx.x % 8 == o serve
// octant o: they draw tickets from that octant's counter; ticket t is tile
// tiles[t % ntiles] of bin f0 + t / ntiles, so every tile's upwind neighbours carry
// smaller tickets and are held by running (or finished) workgroups.  Completion
// is published per tile with the sweep's epoch (agent-scope release).
//
// Every value that decides the loop's course (the ticket, the bin's frozen flag, the
// tile, the parity) is taken into a scalar register.  Held in vector registers they
// make the loop divergent as far as the compiler can tell, and it may then let the
// lanes of one wave run different iterations: lanes 1..63 of wave 0 pass the
// barriers of the next iteration (re-reading the old ticket) while lane 0 waits to
// draw the new one, and the workgroup sweeps the same tile forever.  Thread 0
// publishes the previous tile and draws the next ticket in one block at the top of
// the loop, so no lane-divergent code sits between a tile's last barrier and the
// next ticket's first.
template <typename Real, bool DFORM>
__global__ void __launch_bounds__(64 * kMaxWaves) sweep_persistent_kernel(SweepArgs<Real> A, DagArgs D)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int s_ticket;
    const int oct = blockIdx.x & 7;
    const int items = D.ntiles * A.nfc;
    const int epoch = __builtin_amdgcn_readfirstlane(D.counter[8]);   // set by dag_begin_kernel
    int done_f = -1, done_tile = -1;   // the tile this workgroup finished last (uniform)
    for (;;) {
        if (threadIdx.x == 0) {
            if (done_tile >= 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(D.done + ((int64_t)done_f * 8 + oct) * D.ntiles + done_tile, epoch,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_ticket = atomicAdd(D.counter + oct, 1);
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();
        if (t < 0 || t >= items) break;
        const int fc = t / D.ntiles;
        const int tile = t - fc * D.ntiles;
        const int f = A.f0 + fc;
        const int frozen = __builtin_amdgcn_readfirstlane(A.frozen[f]);
        const int packed = __builtin_amdgcn_readfirstlane(A.tiles[tile]);
        const int par = __builtin_amdgcn_readfirstlane(A.parity[f]);
        done_tile = -1;
        if (frozen | (packed < 0) | (par < 0)) continue;
        sweep_tile<Real, DFORM, true, 1, true, 0>(A, oct, f, packed, par, lds_raw, D.done, epoch, D.ntiles, D.nt0,
                                                  D.nt1, D.err, D.wait_ticks);
        // every wave waits for its own stores of the tile to complete before the
        // barrier; thread 0 then publishes the tile behind one agent-scope release
        // fence (at the top of the loop), which covers the whole workgroup's stores
        tile_stores_done();
        __syncthreads();
        done_f = f;
        done_tile = D.tile_id(packed & 1023, (packed >> 10) & 1023, (packed >> 20) & 1023);
    }
}

// Before a batched persistent sweep: zero the octants' ticket counters of the batch,
// advance the epoch of every member (each member's completion flags carry its own
// epochs, also those of its single solves).
__global__ void dag_begin_batch_kernel(int *counter, const PersistMember *mem, int nmem)
{
    if (blockIdx.x == 0 && threadIdx.x < 8) counter[threadIdx.x] = 0;
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j < nmem) mem[j].counter[8] += 1;
}

// Formal solutions of all members of a batch class in one launch (bins and problems
// are independent, section 3.1).  The work items are listed stage by stage: every
// tile with tx + ty + tz = s of every member and bin comes before any tile of stage
// s + 1, so a tile's upwind neighbours (same member, bin and octant, stage s - 1)
// always carry smaller tickets.  Otherwise the loop is the single-problem one: the
// workgroups of octant o draw tickets from counter[o], wait on the member's
// completion flags, and publish each finished tile with the member's epoch.
template <typename Real, bool DFORM>
__global__ void __launch_bounds__(64 * kMaxWaves)
    sweep_persistent_batch_kernel(const SweepArgs<Real> *args, const PersistMember *mem, const PersistItem *items,
                                  int nitems, int *counter, int *err, uint64_t wait_ticks)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int s_ticket;
    const int oct = blockIdx.x & 7;
    int *pub = nullptr;      // completion flag of the tile this workgroup finished last
    int pub_epoch = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            if (pub) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(pub, pub_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_ticket = atomicAdd(counter + oct, 1);
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_ticket);
        __syncthreads();
        if (t < 0 || t >= nitems) break;
        const int j = __builtin_amdgcn_readfirstlane(items[t].member);
        const int f = __builtin_amdgcn_readfirstlane(items[t].f);
        const int z = __builtin_amdgcn_readfirstlane(items[t].tile);
        const SweepArgs<Real> &A = args[j];
        const PersistMember &M = mem[j];
        const int frozen = __builtin_amdgcn_readfirstlane(A.frozen[f]);
        const int packed = __builtin_amdgcn_readfirstlane(A.tiles[z]);
        const int par = __builtin_amdgcn_readfirstlane(A.parity[f]);
        const int epoch = __builtin_amdgcn_readfirstlane(M.counter[8]);
        pub = nullptr;
        if (frozen | (packed < 0) | (par < 0)) continue;
        sweep_tile<Real, DFORM, true, 1, true, 0>(A, oct, f, packed, par, lds_raw, M.done, epoch, M.ntiles, M.nt0,
                                                  M.nt1, err, wait_ticks);
        tile_stores_done();
        __syncthreads();
        const int tid = (((packed >> 20) & 1023) * M.nt1 + ((packed >> 10) & 1023)) * M.nt0 + (packed & 1023);
        pub = M.done + ((int64_t)f * 8 + oct) * M.ntiles + tid;
        pub_epoch = epoch;
    }
}

// ---- Lambda*: diagonal of the formal-solution operator (section 3.4) -----------------
// Lambda*_ii = sum_k w_k psi0_k: the weight of S at the vertex itself in its own
// update.  psi0 depends only on the upwind chi, so this is a pointwise kernel.  In the
// second-order form the weight taken is beta_k, the coefficient of S0 itself; the
// control point's share gamma_k is left out (it enters only through the clamped
// parabola and makes the Jacobi iteration cycle where the clamp switches).
__global__ void lambda_star_kernel(int nx, int ny, int nz, int px, int py, int pz, int nf, int na, int order,
                                   const RayGeo *rays, const double *chi, double *lam)
{
    const int64_t cells = (int64_t)nx * ny * nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * nf) return;
    const int f = (int)(i / cells);
    const int64_t cc = i - (int64_t)f * cells;
    const int x = (int)(cc % nx), y = (int)((cc / nx) % ny), z = (int)(cc / ((int64_t)nx * ny));
    const double *cf = chi + (int64_t)f * cells;
    const double c0 = cf[cc];
    double acc = 0.0;
    for (int k = 0; k < na; ++k) {
        const RayGeo *G = rays + k;
        const int d = G->d, a = G->a;
        const int sx = (G->oct & 1) ? -1 : 1, sy = (G->oct & 2) ? -1 : 1, sz = (G->oct & 4) ? -1 : 1;
        double cm = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int oa = v & 1, ob = v >> 1;
            // upwind offset along each axis: 1 on d, oa on a, ob on b (times the sign)
            const int ox = d == 0 ? 1 : (a == 0 ? oa : ob);
            const int oy = d == 1 ? 1 : (a == 1 ? oa : ob);
            const int oz = d == 2 ? 1 : (a == 2 ? oa : ob);
            const int ux = fold(x - ox * sx, nx, px), uy = fold(y - oy * sy, ny, py), uz = fold(z - oz * sz, nz, pz);
            cm += G->w4[v] * cf[((int64_t)uz * ny + uy) * nx + ux];
        }
        const double dt = 0.5 * G->s * (cm + c0);
        double E, pm, p0;
        if (order) {
            double ga;
            bezier_coeffs(dt, E, pm, p0, ga);
        } else {
            seg_coeffs(dt, E, pm, p0);
        }
        acc += G->wk * p0;
    }
    lam[i] = acc;
}

template <typename Real>
__global__ void periodic_cold_kernel(SweepArgs<Real> A, int q)
{
    // the periodic slot read next (parity[f]) holds S of the wrapped vertex
    const int64_t P = sel3(q, A.plane[0], A.plane[1], A.plane[2]);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ray = blockIdx.y;
    const int f = blockIdx.z;
    if (i >= P) return;
    const int oct = A.rays[ray].oct;
    // flipped coordinates of the outgoing-plane vertex: coordinate n_q - 1 along q
    const int n1 = (q == 0) ? A.n[1] : A.n[0];
    const int u1 = (int)(i % n1), u2 = (int)(i / n1);
    const int vx = (q == 0) ? A.n[0] - 1 : u1;
    const int vy = (q == 1) ? A.n[1] - 1 : (q == 0 ? u1 : u2);
    const int vz = (q == 2) ? A.n[2] - 1 : u2;
    const int rx = to_real(vx, (oct & 1) ? -1 : 1, A.n[0]);
    const int ry = to_real(vy, (oct & 2) ? -1 : 1, A.n[1]);
    const int rz = to_real(vz, (oct & 4) ? -1 : 1, A.n[2]);
    const double Sv = A.S[(int64_t)f * A.cells + ((int64_t)rz * A.n[1] + ry) * A.n[0] + rx];
    double *Wq = (q == 0) ? A.wrap[0] : (q == 1 ? A.wrap[1] : A.wrap[2]);
    Wq[(((int64_t)f * A.na + ray) * 2 + A.parity[f]) * P + i] = Sv;
}

// Entries of the padded face planes along axis q that hold ghost vertices: the
// whole slot-0 plane and, in each further slot, the row and column at -1.
template <typename Real>
__device__ __forceinline__ int64_t ghost_count(const SweepArgs<Real> &A, int q)
{
    const int na_ = (q == 0) ? A.n[1] : A.n[0], nb_ = (q == 2) ? A.n[1] : A.n[2];
    return (int64_t)(na_ + 1) * (nb_ + 1) + (int64_t)(sel3(q, A.nt[0], A.nt[1], A.nt[2]) - 1) * (na_ + nb_ + 1);
}

// Ghost values of one sweep (section 3.3 boundary conditions: vacuum, thermal,
// given incident intensity, periodic memory) written where the tiles read them.
// blockIdx.y: ray, blockIdx.z: bin - f0.
template <typename Real, bool DFORM>
__device__ __forceinline__ void ghost_fill_one(const SweepArgs<Real> &A, int oct, int f, int e)
{
    // entries of one ray's planes stay far below 2^31 (32-bit index arithmetic)
    if (A.frozen[f]) return;
    int q = 0;
    int cq = (int)ghost_count(A, 0);
    if (e < 0) return;
    if (e >= cq) {
        e -= cq;
        q = 1;
        cq = (int)ghost_count(A, 1);
        if (e >= cq) {
            e -= cq;
            q = 2;
            if (e >= (int)ghost_count(A, 2)) return;
        }
    }
    const int na_ = (q == 0) ? A.n[1] : A.n[0], nb_ = (q == 2) ? A.n[1] : A.n[2];
    const int P0 = (na_ + 1) * (nb_ + 1);
    int t, ia, ib;
    if (e < P0) {
        t = 0;
        ia = e % (na_ + 1) - 1;
        ib = e / (na_ + 1) - 1;
    } else {
        const int e2 = e - P0;
        const int L = na_ + nb_ + 1;
        t = 1 + e2 / L;
        const int k = e2 % L;
        ia = (k <= nb_) ? -1 : k - nb_ - 1;
        ib = (k <= nb_) ? k - 1 : -1;
    }
    const int vq = t * T - 1;
    const int vx = (q == 0) ? vq : ia;
    const int vy = (q == 1) ? vq : (q == 0 ? ia : ib);
    const int vz = (q == 2) ? vq : ib;
    TileCtx c;
    c.f = f;
    c.par = A.parity[f];
    c.fbase = (int64_t)f * A.cells;
    c.sgx = (oct & 1) ? -1 : 1;
    c.sgy = (oct & 2) ? -1 : 1;
    c.sgz = (oct & 4) ? -1 : 1;
    const int ntq = sel3(q, A.nt[0], A.nt[1], A.nt[2]);
    Real *Fq = (q == 0) ? A.face[0] : (q == 1 ? A.face[1] : A.face[2]);
    const FacePlane F(na_, nb_);
    const int64_t slot = sel3(q, A.pplane[0], A.pplane[1], A.pplane[2]);
    const int64_t pos = (int64_t)t * slot + F.at(ia, ib);
    // slot 0 inside the grid: a full block's last column also goes to its copy
    const bool copy = ia >= 0 && ib >= 0 && (ia & (T - 1)) == T - 1;
    const int64_t cpos = (int64_t)t * slot + (copy ? F.col(ia, ib) : 0);
    // S of the folded vertex is the same for every ray of the octant: loaded once
    double Sg = 0.0;
    for (int r = 0; r < A.R; ++r) {
        const int ray = oct * A.R + r;
        const double *src;
        int64_t scell;
        ghost_source(A, c, vx, vy, vz, ray, A.rays[ray].gidx, src, scell);
        if (DFORM && r == 0) Sg = A.S[scell];
        const double I = src ? *src : 0.0;
        const Real v = DFORM ? Real(I - Sg) : Real(I);
        Real *base = Fq + ((int64_t)f * A.na + ray) * ntq * slot;
        base[pos] = v;
        if (copy) base[cpos] = v;
    }
}

template <typename Real>
__device__ __forceinline__ int64_t ghost_total(const SweepArgs<Real> &A)
{
    return ghost_count(A, 0) + ghost_count(A, 1) + ghost_count(A, 2);
}

// blockIdx.y: octant, blockIdx.z: bin - f0; a thread writes its entry for every ray
// of the octant.
template <typename Real, bool DFORM>
__global__ void ghost_fill_kernel(SweepArgs<Real> A)
{
    ghost_fill_one<Real, DFORM>(A, blockIdx.y, A.f0 + (int)blockIdx.z, (int)(blockIdx.x * blockDim.x + threadIdx.x));
}

// Batched form: blockIdx.z is the problem, blockIdx.y the octant, x the entries; each
// thread fills its entry for every bin and every ray of the octant.
template <typename Real, bool DFORM>
__global__ void ghost_fill_batch_kernel(const SweepArgs<Real> *args)
{
    const SweepArgs<Real> &A = args[blockIdx.z];
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= (int)ghost_total(A)) return;
    for (int f = 0; f < A.nf; ++f) ghost_fill_one<Real, DFORM>(A, blockIdx.y, f, e);
}

template <typename Real, int NP>
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
    for (int o = 0; o < NP; ++o) acc += (double)part[o * stride + i];
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
// without cancellation.  Each block writes its max to blockmax (no atomics).  NP
// partial-sum slots (8 octants, or octant x first-crossed axis) are summed in order.
template <typename Real, int NP = 8>
__device__ __forceinline__ void ali_update_body(const Real *part, int dform, int nf, int64_t cells, const double *B,
                                                const double *eps, const double *lam, double *S64, double *Jout,
                                                const AliCtl &ctl, int f)
{
    __shared__ unsigned long long red[4];
    if (ctl.frozen[f]) return;
    const int64_t stride = (int64_t)nf * cells;
    unsigned long long rb = 0ull;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)ctl.nblk * blockDim.x) {
        const int64_t i = (int64_t)f * cells + c;
        double sum = 0.0;
#pragma unroll
        for (int o = 0; o < NP; ++o) sum += (double)part[o * stride + i];
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
        const double r = (Sn != 0.0) ? fabs(dS) / fabs(Sn) : 0.0;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(r);
        rb = bits > rb ? bits : rb;
    }
    rb = wave_max_u64(rb);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rb;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] > m ? red[w] : m;
        ctl.blockmax[(int64_t)f * ctl.nblk + blockIdx.x] = m;
    }
}

template <typename Real, int NP>
__global__ void __launch_bounds__(256) ali_update_kernel(const Real *part, int dform, int nf, int64_t cells,
                                                         const double *B, const double *eps,
                                                         const double *lam, double *S64, double *Jout, AliCtl ctl)
{
    ali_update_body<Real, NP>(part, dform, nf, cells, B, eps, lam, S64, Jout, ctl, blockIdx.y);
}

// Batched form: blockIdx.z is the problem, blockIdx.y the bin, x the ctl.nblk blocks.
template <typename Real>
__global__ void __launch_bounds__(256) ali_update_batch_kernel(const BatchUpdate *bu)
{
    const BatchUpdate &U = bu[blockIdx.z];
    if ((int)blockIdx.y >= U.nf || (int)blockIdx.x >= U.ctl.nblk) return;
    ali_update_body<Real>(static_cast<const Real *>(U.part), U.dform, U.nf, U.cells, U.B, U.eps, U.lam, U.S64, U.J,
                          U.ctl, blockIdx.y);
}

// Per-bin convergence test (eq. conv) after an update: reduce the block maxima,
// count the iteration, flip the periodic slot, freeze converged bins.
__device__ __forceinline__ void ali_finalize_body(const AliCtl &ctl, int nf, double delta_c, int per_bin_stop,
                                                  int fixed_mode)
{
    __shared__ unsigned long long red[4];
    __shared__ int s_all_conv, s_nonfinite, s_active;
    if (threadIdx.x == 0) {
        s_all_conv = 1;
        s_nonfinite = 0;
        s_active = 0;
    }
    __syncthreads();
    for (int f = 0; f < nf; ++f) {
        // uniform across the block, and held in a scalar register so that the compiler
        // keeps the loop (which has barriers) uniform too
        if (__builtin_amdgcn_readfirstlane(ctl.frozen[f])) continue;
        unsigned long long m = 0ull;
        for (int k = threadIdx.x; k < ctl.nblk; k += blockDim.x) {
            const unsigned long long v = ctl.blockmax[(int64_t)f * ctl.nblk + k];
            m = v > m ? v : m;
        }
        m = wave_max_u64(m);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] > m ? red[w] : m;
            m = red[0] > m ? red[0] : m;
            const double r = __longlong_as_double((long long)m);
            ctl.iters[f] += 1;
            ctl.resid[f] = r;
            ctl.parity[f] ^= 1;
            if (!(r <= 1.7976931348623157e308)) s_nonfinite = 1;
            const int conv = r <= delta_c;
            s_all_conv &= conv;
            s_active += 1;
            if (per_bin_stop && conv && !fixed_mode) ctl.frozen[f] = 1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (!per_bin_stop && !fixed_mode && s_active > 0 && s_all_conv)
            for (int f = 0; f < nf; ++f) ctl.frozen[f] = 1;
        int stopped = 1;
        for (int f = 0; f < nf; ++f) stopped &= ctl.frozen[f] != 0;
        ctl.flags[0] = stopped;
        if (s_nonfinite) {
            ctl.flags[1] = 1;
            for (int f = 0; f < nf; ++f) ctl.frozen[f] = 1;
            ctl.flags[0] = 1;
        }
    }
}

__global__ void __launch_bounds__(256) ali_finalize_kernel(AliCtl ctl, int nf, double delta_c, int per_bin_stop,
                                                           int fixed_mode)
{
    ali_finalize_body(ctl, nf, delta_c, per_bin_stop, fixed_mode);
}

// Batched form: one block per problem; the problem's stop flags are also copied into
// done[2 p], done[2 p + 1] so the host reads one array for the whole batch.
__global__ void __launch_bounds__(256) ali_finalize_batch_kernel(const BatchUpdate *bu, int *done)
{
    const BatchUpdate &U = bu[blockIdx.x];
    ali_finalize_body(U.ctl, U.nf, U.delta_c, U.per_bin_stop, U.fixed_mode);
    __syncthreads();
    if (threadIdx.x == 0) {
        done[2 * blockIdx.x] = U.ctl.flags[0];
        done[2 * blockIdx.x + 1] = U.ctl.flags[1];
    }
}

__global__ void flip_parity_kernel(int *parity, const int *frozen, int f0, int cnt)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < cnt && !frozen[f0 + k]) parity[f0 + k] ^= 1;
}

__global__ void convert_f32_kernel(const double *src, float *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

// caller arrays given in FP32 (rt_problem_desc::in_dtype) widened to the library's FP64
__global__ void convert_f64_kernel(const float *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i];
}

__global__ void warm_start_kernel(const double *B, const double *eps, const double *J, double *S, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) S[i] = eps[i] * B[i] + (1.0 - eps[i]) * J[i];
}

// ---- moments epilogue (section 3.2 eqs. Jsum/Hsum/Ksum, section 4) -------------------
// Per-octant partials of w I, w mu_i I, w mu_i mu_j I are summed in fixed octant
// order; the difference form adds S times the angle set's own sums (1, sum w mu_i,
// sum w mu_i mu_j).  tmp holds [10][nfc][cells] for the Q and integration kernels.
template <typename Real, int NP>
__global__ void moments_combine_kernel(const Real *part, const double *S, int dform, int f0, int nfc, int nf,
                                       int64_t cells, MomConst mc, double *J, double *H, double *K, double *tmp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * nfc) return;
    const int fl = (int)(i / cells);
    const int64_t c = i - (int64_t)fl * cells;
    const int f = f0 + fl;
    const double Sv = dform ? S[(int64_t)f * cells + c] : 0.0;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        double acc = 0.0;
#pragma unroll
        for (int o = 0; o < NP; ++o) acc += (double)part[(((int64_t)o * 10 + q) * nfc + fl) * cells + c];
        if (dform) acc = (q == 0) ? Sv + acc : acc + Sv * mc.m[q];
        tmp[((int64_t)q * nfc + fl) * cells + c] = acc;
        if (q == 0 && J) J[(int64_t)f * cells + c] = acc;
        if (q >= 1 && q <= 3 && H) H[((int64_t)(q - 1) * nf + f) * cells + c] = acc;
        if (q >= 4 && K) K[((int64_t)(q - 4) * nf + f) * cells + c] = acc;
    }
}

// d/dq of a field F at index i along an axis of n points (stride st, spacing h):
// central, wrapped when periodic, second-order one-sided at other faces.
__device__ __forceinline__ double axis_deriv(const double *F, int64_t base, int i, int n, int64_t st, double h,
                                             int periodic)
{
    if (n == 1) return 0.0;
    if (periodic) {
        const int ip = (i + 1 == n) ? 0 : i + 1, im = (i == 0) ? n - 1 : i - 1;
        return (F[base + ip * st] - F[base + im * st]) / (2.0 * h);
    }
    if (n == 2) return (F[base + 1 * st] - F[base]) / h;
    if (i == 0) return (-3.0 * F[base] + 4.0 * F[base + st] - F[base + 2 * st]) / (2.0 * h);
    if (i == n - 1)
        return (3.0 * F[base + (int64_t)(n - 1) * st] - 4.0 * F[base + (int64_t)(n - 2) * st] +
                F[base + (int64_t)(n - 3) * st]) / (2.0 * h);
    return (F[base + (int64_t)(i + 1) * st] - F[base + (int64_t)(i - 1) * st]) / (2.0 * h);
}

// Q_nu = 4 pi eps chi (J - B) where chi dx_min <= 1, else -4 pi div H.
__global__ void moments_q_kernel(const double *tmp, int f0, int nfc, int64_t cells, int nx, int ny, int nz, double hx,
                                 double hy, double hz, int px, int py, int pz, double hmin, const double *chi,
                                 const double *eps, const double *B, double *Qt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cells * nfc) return;
    const int fl = (int)(i / cells);
    const int64_t c = i - (int64_t)fl * cells;
    const int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
    const double *Hx = tmp + ((int64_t)1 * nfc + fl) * cells;
    const double *Hy = tmp + ((int64_t)2 * nfc + fl) * cells;
    const double *Hz = tmp + ((int64_t)3 * nfc + fl) * cells;
    double div = 0.0;
    div += axis_deriv(Hx, c - x, x, nx, 1, hx, px);
    div += axis_deriv(Hy, c - (int64_t)y * nx, y, ny, nx, hy, py);
    div += axis_deriv(Hz, c - (int64_t)z * nx * ny, z, nz, (int64_t)nx * ny, hz, pz);
    const int64_t g = (int64_t)(f0 + fl) * cells + c;
    const double fourpi = 4.0 * 3.14159265358979323846;
    const double J = tmp[((int64_t)0 * nfc + fl) * cells + c];
    const double q_int = fourpi * eps[g] * chi[g] * (J - B[g]);
    const double q_dif = -fourpi * div;
    Qt[(int64_t)fl * cells + c] = (chi[g] * hmin <= 1.0) ? q_int : q_dif;
}

// Frequency integrals sum_nu w_nu X_nu, bins added in their order.
__global__ void moments_integrate_kernel(const double *tmp, const double *Qt, const double *w_nu, int f0, int nfc,
                                         int64_t cells, int first, double *J_int, double *H_int, double *K_int,
                                         double *Q_int)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    double acc[11];
#pragma unroll
    for (int q = 0; q < 11; ++q) acc[q] = 0.0;
    for (int fl = 0; fl < nfc; ++fl) {
        const double w = w_nu[f0 + fl];
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] += w * tmp[((int64_t)q * nfc + fl) * cells + c];
        if (Q_int) acc[10] += w * Qt[(int64_t)fl * cells + c];
    }
    if (J_int) J_int[c] = first ? acc[0] : J_int[c] + acc[0];
    if (H_int)
        for (int q = 0; q < 3; ++q) H_int[q * cells + c] = first ? acc[1 + q] : H_int[q * cells + c] + acc[1 + q];
    if (K_int)
        for (int q = 0; q < 6; ++q) K_int[q * cells + c] = first ? acc[4 + q] : K_int[q * cells + c] + acc[4 + q];
    if (Q_int) Q_int[c] = first ? acc[10] : Q_int[c] + acc[10];
}

__global__ void eddington_kernel(const double *J_int, const double *K_int, int64_t cells, double *f_int)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    const double J = J_int[c];
#pragma unroll
    for (int q = 0; q < 6; ++q) f_int[q * cells + c] = (J != 0.0) ? K_int[q * cells + c] / J : 0.0;
}

// Deterministic FP64 sum: per-block sums (fixed tree), then one thread in block order.
__global__ void __launch_bounds__(256) block_sum_kernel(const double *x, int64_t n, double *partial)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void final_sum_kernel(const double *partial, int nblk, double scale, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += partial[b];
    *out = acc * scale;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t sweep_lds_bytes(int real_bytes, int waves, int nq, bool multi, int order)
{
    const size_t staged = order ? (size_t)stage_cells<1>() : (size_t)stage_cells<0>();
    return (size_t)waves * GEO_BYTES + sizeof(double) * staged +
           (size_t)real_bytes * (staged + (size_t)waves * (size_t)wave_lds(nq, multi));
}

template <typename Real, bool DFORM, int NQ, int ORD>
static void launch_stage_ord(const SweepArgs<Real> &A, int waves, hipStream_t st)
{
    const bool multi = A.R > waves;
    const size_t lds = sweep_lds_bytes((int)sizeof(Real), waves, NQ, multi, ORD);
    if constexpr (NQ == 1 && ORD == 0) {
        if (A.noct == 4) {
            dim3 grid4((unsigned)A.stage_cnt * 4u, (unsigned)A.nfc);
            if (multi)
                hipLaunchKernelGGL((sweep_stage_kernel<Real, DFORM, 1, true, 0, 4>), grid4, dim3(64 * waves), lds, st,
                                   A);
            else
                hipLaunchKernelGGL((sweep_stage_kernel<Real, DFORM, 1, false, 0, 4>), grid4, dim3(64 * waves), lds,
                                   st, A);
            return;
        }
    }
    dim3 grid((unsigned)A.stage_cnt * 8u, (unsigned)A.nfc);
    if (multi)
        hipLaunchKernelGGL((sweep_stage_kernel<Real, DFORM, NQ, true, ORD>), grid, dim3(64 * waves), lds, st, A);
    else
        hipLaunchKernelGGL((sweep_stage_kernel<Real, DFORM, NQ, false, ORD>), grid, dim3(64 * waves), lds, st, A);
}

template <typename Real, bool DFORM, int NQ>
static void launch_stage(const SweepArgs<Real> &A, int waves, hipStream_t st)
{
    if (A.order)
        launch_stage_ord<Real, DFORM, NQ, 1>(A, waves, st);
    else
        launch_stage_ord<Real, DFORM, NQ, 0>(A, waves, st);
}

hipError_t launch_sweep_stage_f64(const SweepArgs<double> &A, int waves, int nq, hipStream_t st)
{
    if (nq == NMOM)
        launch_stage<double, false, NMOM>(A, waves, st);
    else
        launch_stage<double, false, 1>(A, waves, st);
    return hipGetLastError();
}

hipError_t launch_sweep_stage_f32(const SweepArgs<float> &A, int waves, int nq, hipStream_t st)
{
    if (nq == NMOM)
        launch_stage<float, true, NMOM>(A, waves, st);
    else
        launch_stage<float, true, 1>(A, waves, st);
    return hipGetLastError();
}

template <typename Real, bool DFORM, int ORD>
static void launch_batch_stage(const SweepArgs<Real> *args, int nprob, int s, int max_items, int waves, bool multi,
                               hipStream_t st)
{
    dim3 grid((unsigned)max_items, (unsigned)nprob);
    const size_t lds = sweep_lds_bytes((int)sizeof(Real), waves, 1, multi, ORD);
    if (multi)
        hipLaunchKernelGGL((sweep_batch_stage_kernel<Real, DFORM, true, ORD>), grid, dim3(64 * waves), lds, st, args, s);
    else
        hipLaunchKernelGGL((sweep_batch_stage_kernel<Real, DFORM, false, ORD>), grid, dim3(64 * waves), lds, st, args, s);
}

hipError_t launch_sweep_batch_stage_f64(const SweepArgs<double> *args, int nprob, int s, int max_items, int waves,
                                        bool multi, int order, hipStream_t st)
{
    if (order)
        launch_batch_stage<double, false, 1>(args, nprob, s, max_items, waves, multi, st);
    else
        launch_batch_stage<double, false, 0>(args, nprob, s, max_items, waves, multi, st);
    return hipGetLastError();
}

hipError_t launch_sweep_batch_stage_f32(const SweepArgs<float> *args, int nprob, int s, int max_items, int waves,
                                        bool multi, int order, hipStream_t st)
{
    if (order)
        launch_batch_stage<float, true, 1>(args, nprob, s, max_items, waves, multi, st);
    else
        launch_batch_stage<float, true, 0>(args, nprob, s, max_items, waves, multi, st);
    return hipGetLastError();
}

template <typename Real, bool DFORM>
static hipError_t launch_persistent(const SweepArgs<Real> &A, const DagArgs &D, int waves, int blocks_per_octant,
                                    hipStream_t st)
{
    hipLaunchKernelGGL((sweep_persistent_kernel<Real, DFORM>), dim3(8u * (unsigned)blocks_per_octant), dim3(64 * waves),
                       sweep_lds_bytes(sizeof(Real), waves, 1, true, 0), st, A, D);
    return hipGetLastError();
}

hipError_t launch_dag_begin(int *counter, hipStream_t st)
{
    hipLaunchKernelGGL(dag_begin_kernel, dim3(1), dim3(64), 0, st, counter);
    return hipGetLastError();
}

hipError_t launch_sweep_persistent_f64(const SweepArgs<double> &A, const DagArgs &D, int waves, int bpo, hipStream_t st)
{
    return launch_persistent<double, false>(A, D, waves, bpo, st);
}

hipError_t launch_sweep_persistent_f32(const SweepArgs<float> &A, const DagArgs &D, int waves, int bpo, hipStream_t st)
{
    return launch_persistent<float, true>(A, D, waves, bpo, st);
}

template <typename Real, bool DFORM>
static hipError_t launch_persistent_batch(const SweepArgs<Real> *args, const PersistMember *mem,
                                          const PersistItem *items, int nitems, int nmem, int *counter, int *err,
                                          uint64_t wait_ticks, int waves, int bpo, hipStream_t st)
{
    hipLaunchKernelGGL(dag_begin_batch_kernel, dim3((unsigned)((nmem + 63) / 64)), dim3(64), 0, st, counter, mem, nmem);
    hipLaunchKernelGGL((sweep_persistent_batch_kernel<Real, DFORM>), dim3(8u * (unsigned)bpo), dim3(64 * waves),
                       sweep_lds_bytes(sizeof(Real), waves, 1, true, 0), st, args, mem, items, nitems, counter, err,
                       wait_ticks);
    return hipGetLastError();
}

hipError_t launch_sweep_persistent_batch_f64(const SweepArgs<double> *args, const PersistMember *mem,
                                             const PersistItem *items, int nitems, int nmem, int *counter, int *err,
                                             uint64_t wait_ticks, int waves, int bpo, hipStream_t st)
{
    return launch_persistent_batch<double, false>(args, mem, items, nitems, nmem, counter, err, wait_ticks, waves,
                                                  bpo, st);
}

hipError_t launch_sweep_persistent_batch_f32(const SweepArgs<float> *args, const PersistMember *mem,
                                             const PersistItem *items, int nitems, int nmem, int *counter, int *err,
                                             uint64_t wait_ticks, int waves, int bpo, hipStream_t st)
{
    return launch_persistent_batch<float, true>(args, mem, items, nitems, nmem, counter, err, wait_ticks, waves, bpo,
                                                st);
}

hipError_t persistent_batch_blocks_per_cu(int real_bytes, int waves, int *blocks)
{
    const size_t lds = sweep_lds_bytes(real_bytes, waves, 1, true, 0);
    if (real_bytes == 8)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_persistent_batch_kernel<double, false>,
                                                            64 * waves, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_persistent_batch_kernel<float, true>, 64 * waves,
                                                        lds);
}

hipError_t persistent_blocks_per_cu(int real_bytes, int waves, int *blocks)
{
    const size_t lds = sweep_lds_bytes(real_bytes, waves, 1, true, 0);
    if (real_bytes == 8)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_persistent_kernel<double, false>, 64 * waves, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, sweep_persistent_kernel<float, true>, 64 * waves, lds);
}

hipError_t launch_lambda_star(const int n[3], const int bc_lo[3], const int bc_hi[3], int nf, int na, int order,
                              const RayGeo *rays, const double *chi, double *lam, hipStream_t st)
{
    (void)bc_hi;  // periodic axes are periodic on both faces
    const int64_t tot = (int64_t)n[0] * n[1] * n[2] * nf;
    hipLaunchKernelGGL(lambda_star_kernel, dim3(blocks_for(tot, 256)), dim3(256), 0, st, n[0], n[1], n[2],
                       (int)(bc_lo[0] == BC_PERIODIC), (int)(bc_lo[1] == BC_PERIODIC), (int)(bc_lo[2] == BC_PERIODIC),
                       nf, na, order, rays, chi, lam);
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
hipError_t launch_ghost_fill(const SweepArgs<Real> &A, hipStream_t st)
{
    int64_t tot = 0;
    for (int q = 0; q < 3; ++q) {
        const int na_ = (q == 0) ? A.n[1] : A.n[0], nb_ = (q == 2) ? A.n[1] : A.n[2];
        tot += (int64_t)(na_ + 1) * (nb_ + 1) + (int64_t)(A.nt[q] - 1) * (na_ + nb_ + 1);
    }
    dim3 grid(blocks_for(tot, 256), 8u, (unsigned)A.nfc);
    constexpr bool dform = sizeof(Real) == 4;   // FP32 sweeps use the difference form
    hipLaunchKernelGGL((ghost_fill_kernel<Real, dform>), grid, dim3(256), 0, st, A);
    return hipGetLastError();
}
template hipError_t launch_ghost_fill<double>(const SweepArgs<double> &, hipStream_t);
template hipError_t launch_ghost_fill<float>(const SweepArgs<float> &, hipStream_t);

template <typename Real>
hipError_t launch_ghost_fill_batch(const SweepArgs<Real> *args, int nprob, int64_t max_entries, int max_na,
                                   hipStream_t st)
{
    (void)max_na;
    dim3 grid(blocks_for(max_entries, 256), 8u, (unsigned)nprob);
    constexpr bool dform = sizeof(Real) == 4;
    hipLaunchKernelGGL((ghost_fill_batch_kernel<Real, dform>), grid, dim3(256), 0, st, args);
    return hipGetLastError();
}
template hipError_t launch_ghost_fill_batch<double>(const SweepArgs<double> *, int, int64_t, int, hipStream_t);
template hipError_t launch_ghost_fill_batch<float>(const SweepArgs<float> *, int, int64_t, int, hipStream_t);

template <typename Real>
hipError_t launch_ali_update_batch(const BatchUpdate *bu, int nprob, int nblk, int max_nf, hipStream_t st)
{
    hipLaunchKernelGGL(ali_update_batch_kernel<Real>, dim3((unsigned)nblk, (unsigned)max_nf, (unsigned)nprob),
                       dim3(256), 0, st, bu);
    return hipGetLastError();
}
template hipError_t launch_ali_update_batch<double>(const BatchUpdate *, int, int, int, hipStream_t);
template hipError_t launch_ali_update_batch<float>(const BatchUpdate *, int, int, int, hipStream_t);

hipError_t launch_ali_finalize_batch(const BatchUpdate *bu, int nprob, int *done, hipStream_t st)
{
    hipLaunchKernelGGL(ali_finalize_batch_kernel, dim3((unsigned)nprob), dim3(256), 0, st, bu, done);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_partial_sum(const Real *part, int npart, const double *S, int dform, int nf, int64_t cells,
                              const int *frozen, double *J, hipStream_t st)
{
    if (npart == kPlaneParts)
        hipLaunchKernelGGL((partial_sum_kernel<Real, kPlaneParts>), dim3(blocks_for(cells * nf, 256)), dim3(256), 0,
                           st, part, S, dform, nf, cells, frozen, J);
    else
        hipLaunchKernelGGL((partial_sum_kernel<Real, 8>), dim3(blocks_for(cells * nf, 256)), dim3(256), 0, st, part,
                           S, dform, nf, cells, frozen, J);
    return hipGetLastError();
}
template hipError_t launch_partial_sum<double>(const double *, int, const double *, int, int, int64_t, const int *,
                                               double *, hipStream_t);
template hipError_t launch_partial_sum<float>(const float *, int, const double *, int, int, int64_t, const int *,
                                              double *, hipStream_t);

template <typename Real>
hipError_t launch_ali_update(const Real *part, int npart, int dform, int nf, int64_t cells, const double *B,
                             const double *eps, const double *lam, double *S64, double *J,
                             AliCtl ctl, hipStream_t st)
{
    dim3 grid((unsigned)ctl.nblk, (unsigned)nf);
    if (npart == kPlaneParts)
        hipLaunchKernelGGL((ali_update_kernel<Real, kPlaneParts>), grid, dim3(256), 0, st, part, dform, nf, cells, B,
                           eps, lam, S64, J, ctl);
    else
        hipLaunchKernelGGL((ali_update_kernel<Real, 8>), grid, dim3(256), 0, st, part, dform, nf, cells, B, eps, lam,
                           S64, J, ctl);
    return hipGetLastError();
}
template hipError_t launch_ali_update<double>(const double *, int, int, int, int64_t, const double *,
                                              const double *, const double *, double *, double *, AliCtl,
                                              hipStream_t);
template hipError_t launch_ali_update<float>(const float *, int, int, int, int64_t, const double *, const double *,
                                             const double *, double *, double *, AliCtl, hipStream_t);

hipError_t launch_ali_finalize(AliCtl ctl, int nf, double delta_c, int per_bin_stop, int fixed_mode,
                               hipStream_t st)
{
    hipLaunchKernelGGL(ali_finalize_kernel, dim3(1), dim3(256), 0, st, ctl, nf, delta_c, per_bin_stop, fixed_mode);
    return hipGetLastError();
}

hipError_t launch_flip_parity(int *parity, const int *frozen, int f0, int cnt, hipStream_t st)
{
    hipLaunchKernelGGL(flip_parity_kernel, dim3(blocks_for(cnt, 64)), dim3(64), 0, st, parity, frozen, f0, cnt);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_moments_combine(const Real *part, int npart, const double *S, int dform, int f0, int nfc, int nf,
                                  int64_t cells, const MomConst &mc, double *J, double *H, double *K, double *tmp,
                                  hipStream_t st)
{
    if (npart == kPlaneParts)
        hipLaunchKernelGGL((moments_combine_kernel<Real, kPlaneParts>), dim3(blocks_for(cells * nfc, 256)), dim3(256), 0,
                           st, part, S, dform, f0, nfc, nf, cells, mc, J, H, K, tmp);
    else
        hipLaunchKernelGGL((moments_combine_kernel<Real, 8>), dim3(blocks_for(cells * nfc, 256)), dim3(256), 0, st,
                           part, S, dform, f0, nfc, nf, cells, mc, J, H, K, tmp);
    return hipGetLastError();
}
template hipError_t launch_moments_combine<double>(const double *, int, const double *, int, int, int, int, int64_t,
                                                   const MomConst &, double *, double *, double *, double *,
                                                   hipStream_t);
template hipError_t launch_moments_combine<float>(const float *, int, const double *, int, int, int, int, int64_t,
                                                  const MomConst &, double *, double *, double *, double *,
                                                  hipStream_t);

hipError_t launch_moments_q(const double *tmp, int f0, int nfc, const int n[3], const double h[3], const int per[3],
                            const double *chi, const double *eps, const double *B, double *Qt, hipStream_t st)
{
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const double hmin = fmin(h[0], fmin(h[1], h[2]));
    hipLaunchKernelGGL(moments_q_kernel, dim3(blocks_for(cells * nfc, 256)), dim3(256), 0, st, tmp, f0, nfc, cells,
                       n[0], n[1], n[2], h[0], h[1], h[2], per[0], per[1], per[2], hmin, chi, eps, B, Qt);
    return hipGetLastError();
}

hipError_t launch_moments_integrate(const double *tmp, const double *Qt, const double *w_nu, int f0, int nfc,
                                    int64_t cells, int first, double *J_int, double *H_int, double *K_int,
                                    double *Q_int, hipStream_t st)
{
    hipLaunchKernelGGL(moments_integrate_kernel, dim3(blocks_for(cells, 256)), dim3(256), 0, st, tmp, Qt, w_nu, f0, nfc,
                       cells, first, J_int, H_int, K_int, Q_int);
    return hipGetLastError();
}

hipError_t launch_eddington(const double *J_int, const double *K_int, int64_t cells, double *f_int, hipStream_t st)
{
    hipLaunchKernelGGL(eddington_kernel, dim3(blocks_for(cells, 256)), dim3(256), 0, st, J_int, K_int, cells, f_int);
    return hipGetLastError();
}

hipError_t launch_sum(const double *x, int64_t n, double scale, double *partial, int nblk, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(block_sum_kernel, dim3((unsigned)nblk), dim3(256), 0, st, x, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(final_sum_kernel, dim3(1), dim3(64), 0, st, partial, nblk, scale, out);
    return hipGetLastError();
}

hipError_t launch_convert_f32(const double *src, float *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(convert_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_convert_f64(const float *src, double *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(convert_f64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_warm_start(const double *B, const double *eps, const double *J, double *S, int64_t n,
                             hipStream_t st)
{
    hipLaunchKernelGGL(warm_start_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, B, eps, J, S, n);
    return hipGetLastError();
}

}  // namespace rtsc
