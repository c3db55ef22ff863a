// Plane-ordered short-characteristics sweep with monotone quadratic interpolation of
// the upwind intensity (section 3.3) for gfx950.
//
// The quadratic stencil of a vertex covers 3 x 3 vertices of the upwind plane, one of
// them on the downwind side of the vertex, so a ray is swept plane by plane along the
// axis its short characteristic crosses first (d): plane t needs only plane t - 1 of
// the same ray, which is complete.  Step t of every ray of every active bin is one
// launch.  A workgroup takes a 16 x 16 tile of plane t for one bin, octant and d
// ("class") and runs the class's rays one after the other: it stages chi and S of the
// tile's upwind window (18 x 18 vertices of plane t - 1) and of its own vertices once,
// then per ray the window of the ray's upwind-plane intensities, and writes the ray's
// new plane and the class's partial sum of w I (or w D; in the moments sweep also
// w mu_i I and w mu_i mu_j I).  Every vertex lies in
// exactly one plane along d, so each class slot of the partial sums is written once
// per sweep: no atomics, and the sum over the slots runs in a fixed order.  Up to
// RMAX rays of a class are staged together, so their window loads go out at once.
//
// Ghost rules (the oracle's): along an in-plane periodic axis the window wraps to
// this sweep's upwind plane; outside a non-periodic in-plane face the upwind side
// takes the face's incoming intensity and the downwind side (an outgoing face)
// repeats the value in line with the vertex.  The plane before the first along d is
// the previous sweep's last plane on a periodic d axis (S of the wrapped vertex
// before any sweep) and the face's incoming intensity otherwise; where several
// non-periodic faces are outside at once, the highest axis gives the intensity.
// chi and S of a ghost are those of the folded (clamped or wrapped) vertex.
//
// The FP32 path keeps D = I - S in the planes; the quadratic interpolation, which is
// not linear, acts on I = D + S formed in FP64 at the nine stencil points, and the
// recurrence is D0 = D- E + (S- - S0) g with D- = I- - S-.  The last plane of a ray
// with a periodic d axis is also kept as I in FP64: the next sweep reads it with its
// own S (which the ALI has changed in between).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rt_device.h"
#include "rt_internal.h"

namespace rtsc {
namespace {

constexpr int PT = kPlaneTile;
constexpr int PW = PT + 2;            // window edge: one vertex on each side of the tile
constexpr int PWIN = PW * PW;
constexpr int RMAX = 4;               // rays of a class staged together

// Monotone quadratic interpolation between f0 (t = 0) and f1 (t = 1) with the third
// point fm at t = -1: the parabola through the three points as a quadratic Bezier
// curve on [0, 1], its control point f0 + (f1 - fm)/4 clamped between f0 and f1.
__device__ __forceinline__ double quad_interp(double fm, double f0, double f1, double t)
{
    double c = f0 + 0.25 * (f1 - fm);
    const double lo = f0 < f1 ? f0 : f1, hi = f0 < f1 ? f1 : f0;
    c = c < lo ? lo : c;
    c = c > hi ? hi : c;
    const double u = 1.0 - t;
    return (u * u * f0 + 2.0 * t * u * c) + t * t * f1;
}

// Where a window entry comes from: in-plane coordinates after wrap / repeat, the
// folded real cell, and, for a boundary ghost, the face giving its intensity.
struct WinSrc {
    int oa, ob;      // flipped in-plane coordinates of the plane value (when face < 0)
    int cell;        // real cell of the folded vertex (chi, S, B)
    int face;        // -1: a plane value; else 2 q + hi of the face giving the intensity
    int fidx;        // index of the folded vertex in that face's plane
};

template <typename Real>
__device__ __forceinline__ WinSrc window_source(const PlaneArgs<Real> &A, int t, int d, int a, int b, int sgd,
                                                int sga, int sgb, int oa, int ob)
{
    const int nd = sel3(d, A.n[0], A.n[1], A.n[2]);
    const int na_ = sel3(a, A.n[0], A.n[1], A.n[2]), nb_ = sel3(b, A.n[0], A.n[1], A.n[2]);
    const int pd_ = sel3(d, A.periodic[0], A.periodic[1], A.periodic[2]);
    const int pa = sel3(a, A.periodic[0], A.periodic[1], A.periodic[2]);
    const int pb = sel3(b, A.periodic[0], A.periodic[1], A.periodic[2]);
    bool ga = false, gb = false, gd = false;
    if (oa < 0) {
        if (pa) oa += na_;
        else { ga = true; oa = 0; }
    } else if (oa >= na_) {
        oa = pa ? oa - na_ : na_ - 1;
    }
    if (ob < 0) {
        if (pb) ob += nb_;
        else { gb = true; ob = 0; }
    } else if (ob >= nb_) {
        ob = pb ? ob - nb_ : nb_ - 1;
    }
    int od = t - 1;
    if (od < 0) {
        if (pd_) od = nd - 1;
        else { gd = true; od = 0; }
    }
    // real coordinates of the folded vertex
    const int rd = to_real(od, sgd, nd), ra = to_real(oa, sga, na_), rb = to_real(ob, sgb, nb_);
    const int rx = d == 0 ? rd : (a == 0 ? ra : rb);
    const int ry = d == 1 ? rd : (a == 1 ? ra : rb);
    const int rz = d == 2 ? rd : (a == 2 ? ra : rb);
    WinSrc w;
    w.oa = oa;
    w.ob = ob;
    w.cell = (rz * A.n[1] + ry) * A.n[0] + rx;
    w.face = -1;
    w.fidx = 0;
    // the highest non-periodic axis among those outside gives the intensity
    int q = -1, sg = 1;
    if (gd && d > q) { q = d; sg = sgd; }
    if (ga && a > q) { q = a; sg = sga; }
    if (gb && b > q) { q = b; sg = sgb; }
    if (q >= 0) {
        const int hi = sg > 0 ? 0 : 1;   // the flipped low side is the real high face for sg < 0
        w.face = 2 * q + hi;
        // index in the plane normal to q: the other two axes in increasing order, lower fastest
        w.fidx = q == 0 ? rz * A.n[1] + ry : (q == 1 ? rz * A.n[0] + rx : ry * A.n[0] + rx);
    }
    return w;
}

// Weight of a ray in accumulated quantity q: w (J), w mu_i (H), w mu_i mu_j (K: xx yy
// zz xy xz yz).
__device__ __forceinline__ double plane_weight(const RayGeo *G, int q)
{
    const double *m = G->mu;
    switch (q) {
    case 0: return G->wk;
    case 1: return G->wk * m[0];
    case 2: return G->wk * m[1];
    case 3: return G->wk * m[2];
    case 4: return G->wk * m[0] * m[0];
    case 5: return G->wk * m[1] * m[1];
    case 6: return G->wk * m[2] * m[2];
    case 7: return G->wk * m[0] * m[1];
    case 8: return G->wk * m[0] * m[2];
    default: return G->wk * m[1] * m[2];
    }
}

// NQ = 1: the class's partial sum of w I (w D); NQ = 10: also w mu_i I and w mu_i mu_j I
// (the moments sweep), slot [class][q].
template <typename Real, bool DFORM, int NQ>
__global__ void __launch_bounds__(PT *PT) plane_step_kernel(PlaneArgs<Real> A, int t)
{
    const int c = blockIdx.y;
    const int oct = c / 3, d = c - 3 * oct;
    const int fl = blockIdx.z, f = A.f0 + fl;
    const int r0 = A.cls_off[c], r1 = A.cls_off[c + 1];
    const int nd = sel3(d, A.n[0], A.n[1], A.n[2]);
    if (r0 == r1 || t >= nd || A.frozen[f] || (int)blockIdx.x >= sel3(d, A.ntiles[0], A.ntiles[1], A.ntiles[2]))
        return;
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    const int na_ = sel3(a, A.n[0], A.n[1], A.n[2]), nb_ = sel3(b, A.n[0], A.n[1], A.n[2]);
    const int tpa = sel3(d, A.tiles_a[0], A.tiles_a[1], A.tiles_a[2]);
    const int a0 = ((int)blockIdx.x % tpa) * PT, b0 = ((int)blockIdx.x / tpa) * PT;
    const int sgx = (oct & 1) ? -1 : 1, sgy = (oct & 2) ? -1 : 1, sgz = (oct & 4) ? -1 : 1;
    const int sgd = sel3(d, sgx, sgy, sgz), sga = sel3(a, sgx, sgy, sgz), sgb = sel3(b, sgx, sgy, sgz);
    const int64_t fbase = (int64_t)f * A.cells;
    const Real *chif = A.chi + fbase;
    const double *Sf = A.S + fbase;
    const double *Bf = A.B + fbase;

    __shared__ double sS[PWIN];      // S of the upwind window (folded vertices)
    __shared__ Real sC[PWIN];        // chi of the upwind window
    __shared__ Real sV[RMAX * PWIN]; // the rays' upwind-plane values (I, or D), one window each
    __shared__ int sSrc[PWIN];       // plane index (>= 0), or -1 - cell of a boundary ghost
    __shared__ int sFace[PWIN], sFidx[PWIN];

    const int tid = threadIdx.x;
    for (int e = tid; e < PWIN; e += PT * PT) {
        const int wx = e % PW, wy = e / PW;
        const WinSrc w = window_source(A, t, d, a, b, sgd, sga, sgb, a0 - 1 + wx, b0 - 1 + wy);
        sS[e] = Sf[w.cell];
        sC[e] = chif[w.cell];
        sFace[e] = w.face;
        sFidx[e] = w.face >= 0 ? w.fidx : w.cell;   // ghosts: the face index; thermal needs the cell
        sSrc[e] = w.face >= 0 ? -1 - w.cell : w.ob * na_ + w.oa;
    }
    // this thread's vertex
    const int ia = a0 + (tid % PT), ib = b0 + (tid / PT);
    const bool act = ia < na_ && ib < nb_;
    int vcell = 0;
    double S0 = 0.0;
    Real C0 = Real(0);
    if (act) {
        const int rd = to_real(t, sgd, nd), ra = to_real(ia, sga, na_), rb = to_real(ib, sgb, nb_);
        const int rx = d == 0 ? rd : (a == 0 ? ra : rb);
        const int ry = d == 1 ? rd : (a == 1 ? ra : rb);
        const int rz = d == 2 ? rd : (a == 2 ? ra : rb);
        vcell = (rz * A.n[1] + ry) * A.n[0] + rx;
        S0 = Sf[vcell];
        C0 = chif[vcell];
    }
    const int par = A.parity[f];
    const int wsel = (t + par * nd) & 1;
    const bool keep_i = DFORM && t == nd - 1 && sel3(d, A.periodic[0], A.periodic[1], A.periodic[2]);
    Real acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = Real(0);
    const int lx = tid % PT + 1, ly = tid / PT + 1;   // the vertex's column in the window
    // up to RMAX rays of the class per pass: all their window loads go out together
    for (int rp = r0; rp < r1; rp += RMAX) {
        const int nr = min(RMAX, r1 - rp);
        int rays[RMAX];
#pragma unroll
        for (int k = 0; k < RMAX; ++k) rays[k] = A.cls_rays[rp + min(k, nr - 1)];
        __syncthreads();   // the previous pass's windows are no longer read
        for (int e = tid; e < PWIN; e += PT * PT) {
            const int src = sSrc[e];
            Real v[RMAX];
            if (src >= 0) {
                // t = 0 reads the previous sweep's last plane (periodic d)
#pragma unroll
                for (int k = 0; k < RMAX; ++k) {
                    const int64_t rb = (int64_t)f * A.na + rays[k];
                    v[k] = (DFORM && t == 0) ? Real(A.wrapI[rb * A.pmax + src] - sS[e])
                                             : A.planes[(rb * 2 + (wsel ^ 1)) * A.pmax + src];
                }
            } else {
                const int face = sFace[e];
                const int kind = (face & 1) ? A.bc_hi[face >> 1] : A.bc_lo[face >> 1];
                const int q = face >> 1;
                const int64_t ps = q == 0 ? (int64_t)A.n[1] * A.n[2]
                                          : (q == 1 ? (int64_t)A.n[0] * A.n[2] : (int64_t)A.n[0] * A.n[1]);
#pragma unroll
                for (int k = 0; k < RMAX; ++k) {
                    double I = 0.0;
                    if (kind == BC_THERMAL)
                        I = Bf[-1 - src];
                    else if (kind == BC_FIXED)
                        I = A.fixed[face][((int64_t)f * A.na + A.rays[rays[k]].gidx) * ps + sFidx[e]];
                    v[k] = DFORM ? Real(I - sS[e]) : Real(I);
                }
            }
#pragma unroll
            for (int k = 0; k < RMAX; ++k) sV[k * PWIN + e] = v[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
            if (k >= nr || !act) continue;
            const int ray = rays[k];
            const RayGeo *G = A.rays + ray;
            const int64_t rb = (int64_t)f * A.na + ray;
            const Real *win = sV + k * PWIN;
            const double fa = G->fa, fb = G->fb;
            auto Iat = [&](int ua, int ub) {
                const int e = (ly - ub) * PW + (lx - ua);
                return DFORM ? double(win[e]) + sS[e] : double(win[e]);
            };
            double row[3];
#pragma unroll
            for (int ub = -1; ub <= 1; ++ub) row[ub + 1] = quad_interp(Iat(-1, ub), Iat(0, ub), Iat(1, ub), fa);
            const double Im = quad_interp(row[0], row[1], row[2], fb);
            // S- and chi- bilinear on the upwind face: offsets (0,0) (1,0) (0,1) (1,1)
            const int e00 = ly * PW + lx, e10 = e00 - 1, e01 = e00 - PW, e11 = e00 - PW - 1;
            const double w00 = G->w4[0], w10 = G->w4[1], w01 = G->w4[2], w11 = G->w4[3];
            const double Sm = ((w00 * sS[e00] + w10 * sS[e10]) + w01 * sS[e01]) + w11 * sS[e11];
            Real v;
            if constexpr (DFORM) {
                const float Cm = float(w00) * sC[e00] + float(w10) * sC[e10] + float(w01) * sC[e01] +
                                 float(w11) * sC[e11];
                const float dt = float(0.5 * G->s) * (Cm + C0);
                float E, g;
                seg_coeffs(dt, E, g);
                const float Dm = float(Im - Sm);
                v = Dm * E + float(Sm - S0) * g;
            } else {
                const double Cm = ((w00 * sC[e00] + w10 * sC[e10]) + w01 * sC[e01]) + w11 * sC[e11];
                const double dt = G->s * (Cm + C0) * 0.5;
                double E, pm, p0;
                seg_coeffs(dt, E, pm, p0);
                v = (Im * E + pm * Sm) + p0 * S0;
            }
            A.planes[(rb * 2 + wsel) * A.pmax + ib * na_ + ia] = v;
            if (keep_i) A.wrapI[rb * A.pmax + ib * na_ + ia] = double(v) + S0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += Real(plane_weight(G, q)) * v;
        }
    }
    if (act) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) A.part[(((int64_t)c * NQ + q) * A.nfc + fl) * A.cells + vcell] = acc[q];
    }
}

// Before the first sweep (and after a reset of the periodic memory) the plane read at
// t = 0 by every ray whose d axis is periodic holds I = S of the wrapped vertex (the
// plane n_d - 1): in the plane slot, or in the FP64 copy of the difference form.
template <typename Real, bool DFORM>
__global__ void plane_cold_kernel(PlaneArgs<Real> A)
{
    const int ray = blockIdx.y, fl = blockIdx.z, f = A.f0 + fl;
    const RayGeo *G = A.rays + ray;
    const int d = G->d, a = G->a, b = G->b;
    if (!sel3(d, A.periodic[0], A.periodic[1], A.periodic[2])) return;
    const int nd = sel3(d, A.n[0], A.n[1], A.n[2]);
    const int na_ = sel3(a, A.n[0], A.n[1], A.n[2]), nb_ = sel3(b, A.n[0], A.n[1], A.n[2]);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)na_ * nb_) return;
    const int oa = (int)(i % na_), ob = (int)(i / na_);
    const int oct = G->oct;
    const int sgx = (oct & 1) ? -1 : 1, sgy = (oct & 2) ? -1 : 1, sgz = (oct & 4) ? -1 : 1;
    const int rd = to_real(nd - 1, sel3(d, sgx, sgy, sgz), nd);
    const int ra = to_real(oa, sel3(a, sgx, sgy, sgz), na_), rb = to_real(ob, sel3(b, sgx, sgy, sgz), nb_);
    const int rx = d == 0 ? rd : (a == 0 ? ra : rb);
    const int ry = d == 1 ? rd : (a == 1 ? ra : rb);
    const int rz = d == 2 ? rd : (a == 2 ? ra : rb);
    const int par = A.parity[f];
    const int rsel = (par * nd & 1) ^ 1;   // the slot step 0 reads
    const double S = A.S[(int64_t)f * A.cells + (rz * A.n[1] + ry) * A.n[0] + rx];
    if (DFORM)
        A.wrapI[((int64_t)f * A.na + ray) * A.pmax + i] = S;
    else
        A.planes[(((int64_t)f * A.na + ray) * 2 + rsel) * A.pmax + i] = Real(S);
}

inline unsigned blocks_of(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <typename Real>
hipError_t launch_plane_step(const PlaneArgs<Real> &A, int t, int nq, hipStream_t st)
{
    const int tiles = std::max(A.ntiles[0], std::max(A.ntiles[1], A.ntiles[2]));
    dim3 grid((unsigned)tiles, (unsigned)kPlaneParts, (unsigned)A.nfc);
    constexpr bool DF = sizeof(Real) == 4;
    if (nq == 10)
        hipLaunchKernelGGL((plane_step_kernel<Real, DF, 10>), grid, dim3(PT * PT), 0, st, A, t);
    else
        hipLaunchKernelGGL((plane_step_kernel<Real, DF, 1>), grid, dim3(PT * PT), 0, st, A, t);
    return hipGetLastError();
}
template hipError_t launch_plane_step<float>(const PlaneArgs<float> &, int, int, hipStream_t);
template hipError_t launch_plane_step<double>(const PlaneArgs<double> &, int, int, hipStream_t);

template <typename Real>
hipError_t launch_plane_cold(const PlaneArgs<Real> &A, hipStream_t st)
{
    dim3 grid(blocks_of(A.pmax, 256), (unsigned)A.na, (unsigned)A.nfc);
    if constexpr (sizeof(Real) == 4)
        hipLaunchKernelGGL((plane_cold_kernel<float, true>), grid, dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL((plane_cold_kernel<double, false>), grid, dim3(256), 0, st, A);
    return hipGetLastError();
}
template hipError_t launch_plane_cold<float>(const PlaneArgs<float> &, hipStream_t);
template hipError_t launch_plane_cold<double>(const PlaneArgs<double> &, hipStream_t);

}  // namespace rtsc
