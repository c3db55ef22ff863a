/*
 * rt_oracle.c -- plain, slow FP64 CPU reference for the short-characteristics
 * formal solution of Davis, Stone & Jiang (2012), "A Radiation Transfer Solver
 * for Athena using Short Characteristics" (arXiv:1201.2222).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link
 * or call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP implementation.
 *
 * What it computes (paper section 3.3, eq. rtdisc, and section 3.2, eqs.
 * Jsum/Hsum/Ksum): for every ray k and every vertex x0 of the radiation grid
 * (vertices = cell centres), the intensity I0 is integrated along the short
 * characteristic from the upwind point x- on the face of the upwind cell box:
 *
 *     I0 = I- exp(-dtau) + psi- S- + psi0 S0                  (first order form)
 *
 * or, in the second-order form of eq. rtdisc with Bezier interpolation of the
 * source function (order = 1), a quadratic Bezier curve in optical depth from S0
 * back to S- whose control point Sc = S0 - dtau-/2 (dS/dtau)0 is clamped to the
 * interval [min(S-, S0), max(S-, S0)] (no overshoot); (dS/dtau)0 is the
 * derivative of the parabola through S-, S0 and the downwind S+ (optical depth
 * intervals dtau- and dtau+), so
 *
 *     I0 = I- exp(-dtau-) + alpha S- + beta S0 + gamma Sc,
 *
 * with alpha, beta, gamma the integrals of exp(-t) against the Bezier basis.
 *
 * where I-, S- and chi- are bilinear interpolants on that face (section 3.3,
 * "first-order (linear) interpolation"), dtau is the trapezoid optical depth of
 * the segment, and psi-, psi0 integrate a source function that is linear in
 * optical depth between S- and S0.  Moments J = sum w I, H_i = sum w mu_i I,
 * K_ij = sum w mu_i mu_j I.  The diagonal of the Lambda operator (section 3.4,
 * eq. dsjacobi) is Lambda_ii = sum_k w_k psi0_k (first order); for the second-order
 * form it is taken as sum_k w_k beta_k, the weight of S0 with the control point held
 * fixed.  The diagonal only sets how the Jacobi iteration approaches its fixed point;
 * counting the control point as S0 too (beta + gamma) overestimates the response
 * where the control point is clamped, and the iteration then cycles between the
 * clamped and unclamped states instead of converging.
 *
 * Sweep order: each ray is swept on its own over the whole grid in row-major
 * order (x fastest) starting from the upwind corner of its octant, the order of
 * the paper's Fig. f:sweep generalised to 3D.  Every upwind vertex then lies
 * earlier in that order, so I- is always known.
 *
 * Upwind intensity (interp): bilinear on the 2 x 2 upwind face (0), or the
 * monotone quadratic interpolation section 3.3 names as the alternative (1): on the
 * 3 x 3 stencil of the upwind plane, each line is interpolated by a quadratic
 * Bezier curve whose control point comes from the parabola through the three
 * points and is clamped between the two bracketing values (orc_quad_interp),
 * along a first and then along b.  Its stencil reaches one vertex past the vertex
 * on the downwind side, so each ray is then swept plane by plane along the axis
 * its characteristic crosses first (the section's reordering of the sweep for the
 * rays that would otherwise be shallow), and in-plane periodic wraps read this
 * sweep's values.  S and chi stay bilinear, so the coefficients and Lambda* are
 * those of the first-order form.
 *
 * Boundaries (section 3.5, and the iteration of section 3 for periodic
 * boundaries): a ghost vertex just outside the grid takes chi and S (and B) from
 * the boundary vertex (periodic axes wrap instead of clamp).  Its intensity is
 *   vacuum  : 0
 *   thermal : B of that boundary vertex
 *   fixed   : a caller-given array
 *   periodic: the intensity the previous sweep produced at the wrapped vertex
 *             ("fixed from the previous iteration"); before any sweep has run,
 *             S of the wrapped vertex.
 * When a ghost vertex lies outside a non-periodic face and another face at the
 * same time, the non-periodic face with the highest axis (z, then y, then x)
 * gives the intensity.
 *
 * The Gauss-Seidel form of the Lambda iteration (section 3.4) is here twice: in the
 * paper's zone order (orc_gs_point_iteration) and with the horizontal planes as the
 * blocks of its ordering (orc_gs_iteration), the variant the GPU library runs.
 *
 * Arithmetic is plain FP64 in the order written; build with
 * -ffp-contract=off so that no multiply-add is fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_VACUUM 0
#define ORC_THERMAL 1
#define ORC_PERIODIC 2
#define ORC_FIXED 3

typedef struct {
    int32_t n[3];      /* nx, ny, nz (x fastest in memory) */
    int32_t nf;        /* frequency bins */
    int32_t na;        /* rays */
    int32_t bc_lo[3];  /* boundary kind at the low face of each axis */
    int32_t bc_hi[3];  /* boundary kind at the high face of each axis */
    int32_t want_hk;   /* non-zero: also accumulate H and K */
    double h[3];       /* dx, dy, dz */
    int32_t order;     /* 0: first order (linear), 1: second order (Bezier) */
    int32_t interp;    /* upwind intensity: 0 bilinear, 1 monotone quadratic (plane order) */
} orc_grid;

/* Per-ray geometry of the upwind short characteristic (section 3.3). */
typedef struct {
    int sgn[3];     /* direction signs, +1 when the cosine is zero */
    int d;          /* axis whose face plane the upwind segment crosses first */
    int a, b;       /* the two other axes, a < b */
    double s;       /* path length from the upwind face point to the vertex */
    double fa, fb;  /* fractional offsets of the face point along a and b */
} orc_ray;

static void ray_geometry(const double mu[3], const double h[3], orc_ray *r)
{
    double len[3];
    for (int q = 0; q < 3; ++q) {
        r->sgn[q] = (mu[q] < 0.0) ? -1 : 1;
        len[q] = (mu[q] == 0.0) ? INFINITY : h[q] / fabs(mu[q]);
    }
    /* the plane reached first going upwind; on equal lengths z wins over y
       and y over x */
    int d = 2;
    if (len[1] < len[d]) d = 1;
    if (len[0] < len[d]) d = 0;
    r->d = d;
    r->a = (d == 0) ? 1 : 0;
    r->b = (d == 2) ? 1 : 2;
    r->s = len[d];
    double fa = r->s * fabs(mu[r->a]) / h[r->a];
    double fb = r->s * fabs(mu[r->b]) / h[r->b];
    r->fa = fa > 1.0 ? 1.0 : fa;
    r->fb = fb > 1.0 ? 1.0 : fb;
}

/*
 * Coefficients of the first-order (linear in tau) integration over one segment
 * of optical depth dt:  I0 = I- E + psim S- + psi0 S0.
 *   E = exp(-dt), e0 = 1 - exp(-dt), psi0 = 1 - e0/dt, psim = e0 - psi0.
 * For small dt, psi0 is summed from its Taylor series
 *   psi0 = sum_{n>=1} (-1)^(n+1) dt^n / (n+1)!
 * to avoid the cancellation in 1 - e0/dt.
 */
void orc_coeffs(double dt, double *E, double *psim, double *psi0)
{
    double e0 = -expm1(-dt);
    double p0;
    if (dt < 0.1) {
        /* terms n = 1..13, summed from the smallest upward */
        double term[14];
        double fact = 1.0; /* (n+1)! */
        double pw = 1.0;   /* dt^n */
        for (int n = 1; n <= 13; ++n) {
            pw *= dt;
            fact *= (double)(n + 1);
            term[n] = ((n % 2) ? pw : -pw) / fact;
        }
        p0 = 0.0;
        for (int n = 13; n >= 1; --n) p0 += term[n];
    } else {
        p0 = 1.0 - e0 / dt;
    }
    *E = exp(-dt);
    *psi0 = p0;
    *psim = e0 - p0;
}

/*
 * Coefficients of the second-order (quadratic Bezier in optical depth) integration
 * over one upwind segment of optical depth dt, t measured from x0 upwind:
 *   S(u) = (1-u)^2 S0 + 2u(1-u) Sc + u^2 S-,  u = t/dt,
 *   I0 = I- E + alpha S- + beta S0 + gamma Sc,
 *   alpha = int_0^dt (t/dt)^2 e^-t dt', gamma = int 2 (t/dt)(1 - t/dt) e^-t,
 *   beta  = int (1 - t/dt)^2 e^-t.
 * With e0 = 1 - e^-dt, e1 = int t e^-t = 1 - e^-dt (1 + dt),
 * e2 = int t^2 e^-t = 2 - e^-dt (dt^2 + 2 dt + 2):
 *   alpha = e2/dt^2, gamma = 2 e1/dt - 2 e2/dt^2, beta = e0 - alpha - gamma.
 * Below dt = 0.5 the three come from their series (n >= 0)
 *   alpha = sum (-1)^n (n+1)(n+2) dt^(n+1) / (n+3)!,
 *   gamma = sum (-1)^n 2(n+1) dt^(n+1) / (n+3)!,
 *   beta  = sum (-1)^n 2 dt^(n+1) / (n+3)!,
 * which avoid the cancellation in e1 and e2 (30 terms, summed from the smallest).
 */
void orc_bezier_coeffs(double dt, double *E, double *alpha, double *beta, double *gamma)
{
    *E = exp(-dt);
    if (dt < 0.5) {
        double ta[30], tb[30], tg[30];
        double pw = 1.0;      /* dt^(n+1) */
        double fact = 6.0;    /* (n+3)! */
        for (int n = 0; n < 30; ++n) {
            pw *= dt;
            if (n > 0) fact *= (double)(n + 3);
            double sg = (n % 2) ? -1.0 : 1.0;
            ta[n] = sg * (double)((n + 1) * (n + 2)) * pw / fact;
            tg[n] = sg * 2.0 * (double)(n + 1) * pw / fact;
            tb[n] = sg * 2.0 * pw / fact;
        }
        double a = 0.0, b = 0.0, c = 0.0;
        for (int n = 29; n >= 0; --n) {
            a += ta[n];
            b += tb[n];
            c += tg[n];
        }
        *alpha = a;
        *beta = b;
        *gamma = c;
        return;
    }
    double e0 = -expm1(-dt);
    double ed = exp(-dt);
    double e1 = 1.0 - ed * (1.0 + dt);
    double e2 = 2.0 - ed * (dt * dt + 2.0 * dt + 2.0);
    *alpha = e2 / (dt * dt);
    *gamma = 2.0 * e1 / dt - 2.0 * e2 / (dt * dt);
    *beta = e0 - *alpha - *gamma;
}

/*
 * Control point of the Bezier source function at x0: Sc = S0 - h1/2 S', with S' the
 * derivative at x0 of the parabola through (-h1, S-), (0, S0), (h2, S+) in optical
 * depth, S' = (h2 d- + h1 d+)/(h1 + h2), d- = (S0 - S-)/h1, d+ = (S+ - S0)/h2;
 * clamped to [min(S-, S0), max(S-, S0)].  Degenerate intervals: with h2 = 0 the
 * one-sided slope d- is used; with h1 = 0 the segment carries no weight and Sc = S0.
 */
double orc_control_point(double Sm, double S0, double Sp, double h1, double h2)
{
    double Sc;
    if (!(h1 > 0.0)) {
        Sc = S0;
    } else if (!(h2 > 0.0)) {
        double dm = (S0 - Sm) / h1;
        Sc = S0 - 0.5 * h1 * dm;
    } else {
        double dm = (S0 - Sm) / h1;
        double dp = (Sp - S0) / h2;
        double Sd = (h2 * dm + h1 * dp) / (h1 + h2);
        Sc = S0 - 0.5 * h1 * Sd;
    }
    double lo = Sm < S0 ? Sm : S0;
    double hi = Sm < S0 ? S0 : Sm;
    if (Sc < lo) Sc = lo;
    if (Sc > hi) Sc = hi;
    return Sc;
}

static inline int is_periodic(const orc_grid *g, int q)
{
    return g->bc_lo[q] == ORC_PERIODIC;
}

/* Bring an index that may be one step outside [0, n) back inside: wrap on a
   periodic axis, clamp otherwise.  *out is set when the index was outside. */
static inline int fold(int x, int n, int periodic, int *out)
{
    if (x >= 0 && x < n) return x;
    *out = 1;
    if (periodic) return (x < 0) ? x + n : x - n;
    return (x < 0) ? 0 : n - 1;
}

static inline int64_t cell_index(const orc_grid *g, int i, int j, int k)
{
    return ((int64_t)k * g->n[1] + j) * g->n[0] + i;
}

/* index inside the plane normal to axis q, with the other two axes in
   increasing order and the lower one fastest */
static inline int64_t plane_index(const orc_grid *g, int q, const int u[3])
{
    int p1 = (q == 0) ? 1 : 0;
    int p2 = (q == 2) ? 1 : 2;
    return (int64_t)u[p2] * g->n[p1] + u[p1];
}

static inline int64_t plane_size(const orc_grid *g, int q)
{
    int p1 = (q == 0) ? 1 : 0;
    int p2 = (q == 2) ? 1 : 2;
    return (int64_t)g->n[p1] * g->n[p2];
}

typedef struct {
    const orc_grid *g;
    int f;                    /* bin */
    int ray;                  /* ray index */
    const double *chi, *S, *B;  /* this bin's fields */
    const double *Icur;       /* this ray's intensities of the current sweep */
    const double *const *fixed;   /* [6]: lo x, hi x, lo y, hi y, lo z, hi z */
    const double *const *prev;    /* [3]: per periodic axis, previous sweep */
    int have_prev;
    const double *Scold;      /* S of the wrapped vertex before any sweep (periodic ghosts) */
} orc_ctx;

/* chi and S at vertex v (possibly a ghost vertex) */
static void vertex_fields(const orc_ctx *c, const int v[3], double *chi, double *S)
{
    int u[3], out = 0;
    for (int q = 0; q < 3; ++q) u[q] = fold(v[q], c->g->n[q], is_periodic(c->g, q), &out);
    int64_t id = cell_index(c->g, u[0], u[1], u[2]);
    *chi = c->chi[id];
    *S = c->S[id];
}

/* intensity of the current ray at vertex v (possibly a ghost vertex) */
static double vertex_intensity(const orc_ctx *c, const int v[3])
{
    const orc_grid *g = c->g;
    int u[3], outq[3] = {0, 0, 0};
    int any = 0;
    for (int q = 0; q < 3; ++q) {
        u[q] = fold(v[q], g->n[q], is_periodic(g, q), &outq[q]);
        any |= outq[q];
    }
    if (!any) return c->Icur[cell_index(g, u[0], u[1], u[2])];

    for (int q = 2; q >= 0; --q) {
        if (!outq[q] || is_periodic(g, q)) continue;
        int hi = v[q] >= g->n[q];
        int kind = hi ? g->bc_hi[q] : g->bc_lo[q];
        if (kind == ORC_VACUUM) return 0.0;
        if (kind == ORC_THERMAL) return c->B[cell_index(g, u[0], u[1], u[2])];
        /* fixed incident intensity: [nf][na][plane] */
        const double *F = c->fixed[2 * q + hi];
        int64_t ps = plane_size(g, q);
        return F[((int64_t)c->f * g->na + c->ray) * ps + plane_index(g, q, u)];
    }
    /* only periodic axes are outside */
    if (!c->have_prev) return c->Scold[cell_index(g, u[0], u[1], u[2])];
    for (int q = 0; q < 3; ++q) {
        if (!outq[q]) continue;
        int64_t ps = plane_size(g, q);
        return c->prev[q][((int64_t)c->f * g->na + c->ray) * ps + plane_index(g, q, u)];
    }
    return 0.0; /* not reached */
}

/*
 * Monotone quadratic interpolation of the upwind intensity (section 3.3 names a
 * monotonic second-order scheme that neither overshoots nor loses positivity).  On
 * one line of the upwind plane, f0 is the value in line with the vertex (t = 0), f1
 * one step upwind (t = 1) and fm one step on the downwind side (t = -1); the point
 * sits at t in [0, 1].  The parabola through the three points equals the quadratic
 * Bezier curve on [0, 1] with control point c = f0 + (f1 - fm)/4; c is clamped to
 * [min(f0, f1), max(f0, f1)], so the result lies between f0 and f1.  Collinear data
 * give c = (f0 + f1)/2, the linear interpolant.
 */
double orc_quad_interp(double fm, double f0, double f1, double t)
{
    double c = f0 + 0.25 * (f1 - fm);
    double lo = f0 < f1 ? f0 : f1;
    double hi = f0 < f1 ? f1 : f0;
    if (c < lo) c = lo;
    if (c > hi) c = hi;
    double u = 1.0 - t;
    return (u * u * f0 + 2.0 * t * u * c) + t * t * f1;
}

/*
 * Intensity at a point of the 3 x 3 stencil on the upwind plane of vertex vc for the
 * quadratic scheme: ua, ub = +1 one step upwind along a, b, 0 in line with the vertex,
 * -1 one step on the downwind side.  The sweep visits whole planes in order along
 * d, so the upwind plane is complete: a wrap along a periodic in-plane axis reads this
 * sweep's value.  Outside a non-periodic in-plane face, the upwind side is the face's
 * incoming boundary intensity and the downwind side (an outgoing face) repeats the
 * value in line with the vertex.  The plane before the first (along d) follows the
 * ghost rules of vertex_intensity: previous sweep on a periodic d axis, boundary
 * intensity otherwise.
 */
static double stencil_intensity(const orc_ctx *c, const orc_ray *r, const int vc[3], int ua, int ub)
{
    const orc_grid *g = c->g;
    int v[3];
    v[r->d] = vc[r->d] - r->sgn[r->d];
    const int ax[2] = {r->a, r->b};
    const int off[2] = {ua, ub};
    for (int k = 0; k < 2; ++k) {
        const int q = ax[k];
        v[q] = vc[q] - off[k] * r->sgn[q];
        if (v[q] >= 0 && v[q] < g->n[q]) continue;
        if (is_periodic(g, q))
            v[q] = (v[q] < 0) ? v[q] + g->n[q] : v[q] - g->n[q];
        else if (off[k] < 0)
            v[q] = vc[q];
    }
    return vertex_intensity(c, v);
}

/* bilinear weights of the upwind face at offsets (0,0) (1,0) (0,1) (1,1) along (a, b) */
static void face_weights(const orc_ray *r, double wv[4])
{
    wv[0] = (1.0 - r->fa) * (1.0 - r->fb);
    wv[1] = r->fa * (1.0 - r->fb);
    wv[2] = (1.0 - r->fa) * r->fb;
    wv[3] = r->fa * r->fb;
}

/*
 * The short characteristic of one ray ending at vertex cpos, with the intensities of
 * the ray's current sweep in c->Icur and the source function c->S: returns I0 and the
 * weight of S0 in it (the ray's share of Lambda*).
 */
static void vertex_solve(const orc_ctx *c, const orc_ray *r, const double wv[4], const int cpos[3], double *I0_out,
                         double *ldiag_out)
{
    static const int oa[4] = {0, 1, 0, 1};
    static const int ob[4] = {0, 0, 1, 1};
    const orc_grid *g = c->g;
    const int i = cpos[0], j = cpos[1], k = cpos[2];
    double Iv[4], Sv[4], Cv[4];
    for (int t = 0; t < 4; ++t) {
        int v[3] = {i, j, k};
        v[r->d] -= r->sgn[r->d];
        v[r->a] -= oa[t] * r->sgn[r->a];
        v[r->b] -= ob[t] * r->sgn[r->b];
        Iv[t] = vertex_intensity(c, v);
        vertex_fields(c, v, &Cv[t], &Sv[t]);
    }
    double Im;
    if (g->interp == 1) {
        /* rows at b offsets -1, 0, +1 (downwind side, vertex, upwind side), each
           interpolated along a, then along b */
        double row[3];
        for (int ub = -1; ub <= 1; ++ub) {
            double f[3];
            for (int ua = -1; ua <= 1; ++ua) f[ua + 1] = stencil_intensity(c, r, cpos, ua, ub);
            row[ub + 1] = orc_quad_interp(f[0], f[1], f[2], r->fa);
        }
        Im = orc_quad_interp(row[0], row[1], row[2], r->fb);
    } else {
        Im = ((wv[0] * Iv[0] + wv[1] * Iv[1]) + wv[2] * Iv[2]) + wv[3] * Iv[3];
    }
    double Sm = ((wv[0] * Sv[0] + wv[1] * Sv[1]) + wv[2] * Sv[2]) + wv[3] * Sv[3];
    double Cm = ((wv[0] * Cv[0] + wv[1] * Cv[1]) + wv[2] * Cv[2]) + wv[3] * Cv[3];
    int64_t id = cell_index(g, i, j, k);
    double S0 = c->S[id];
    double dt = r->s * (Cm + c->chi[id]) * 0.5;
    double I0, ldiag;
    if (g->order == 1) {
        /* downwind point: the mirror image of the upwind one */
        double Sp4[4], Cp4[4];
        for (int t = 0; t < 4; ++t) {
            int v[3] = {i, j, k};
            v[r->d] += r->sgn[r->d];
            v[r->a] += oa[t] * r->sgn[r->a];
            v[r->b] += ob[t] * r->sgn[r->b];
            vertex_fields(c, v, &Cp4[t], &Sp4[t]);
        }
        double Sp = ((wv[0] * Sp4[0] + wv[1] * Sp4[1]) + wv[2] * Sp4[2]) + wv[3] * Sp4[3];
        double Cp = ((wv[0] * Cp4[0] + wv[1] * Cp4[1]) + wv[2] * Cp4[2]) + wv[3] * Cp4[3];
        double dtp = r->s * (c->chi[id] + Cp) * 0.5;
        double Sc = orc_control_point(Sm, S0, Sp, dt, dtp);
        double E, al, be, ga;
        orc_bezier_coeffs(dt, &E, &al, &be, &ga);
        I0 = ((Im * E + al * Sm) + be * S0) + ga * Sc;
        ldiag = be;
    } else {
        double E, psim, psi0;
        orc_coeffs(dt, &E, &psim, &psi0);
        I0 = (Im * E + psim * Sm) + psi0 * S0;
        ldiag = psi0;
    }
    *I0_out = I0;
    *ldiag_out = ldiag;
}

/* keep one ray's intensity on its outgoing plane of every periodic axis for the
   next sweep */
static void save_periodic(const orc_grid *g, const orc_ray *r, int f, int ray, const double *Icur,
                          double *const *prev_out)
{
    for (int q = 0; q < 3; ++q) {
        if (!is_periodic(g, q) || !prev_out || !prev_out[q]) continue;
        int64_t ps = plane_size(g, q);
        double *P = prev_out[q] + ((int64_t)f * g->na + ray) * ps;
        int u[3];
        for (u[2] = 0; u[2] < g->n[2]; ++u[2])
            for (u[1] = 0; u[1] < g->n[1]; ++u[1])
                for (u[0] = 0; u[0] < g->n[0]; ++u[0]) {
                    int outc = (r->sgn[q] > 0) ? g->n[q] - 1 : 0;
                    if (u[q] != outc) continue;
                    P[plane_index(g, q, u)] = Icur[cell_index(g, u[0], u[1], u[2])];
                }
    }
}

/* visiting order of a ray: row-major from the upwind corner (x fastest), or, for the
   quadratic upwind intensity, plane by plane along d; idx -> real coordinates */
static void visit_position(const orc_grid *g, const orc_ray *r, int64_t idx, int cpos[3])
{
    int ol[3];
    if (g->interp == 1) {
        const int64_t per = (int64_t)g->n[r->a] * g->n[r->b];
        ol[r->d] = (int)(idx / per);
        ol[r->a] = (int)((idx % per) % g->n[r->a]);
        ol[r->b] = (int)((idx % per) / g->n[r->a]);
    } else {
        ol[0] = (int)(idx % g->n[0]);
        ol[1] = (int)((idx / g->n[0]) % g->n[1]);
        ol[2] = (int)(idx / ((int64_t)g->n[0] * g->n[1]));
    }
    for (int q = 0; q < 3; ++q) cpos[q] = (r->sgn[q] > 0) ? ol[q] : g->n[q] - 1 - ol[q];
}

/*
 * One formal solution: every ray swept once over every bin.
 *   mu  [na][3] direction cosines, w [na] weights (summing to 1)
 *   chi, B, S  [nf][nz][ny][nx]
 *   fixed[6]   incident intensity per face ([nf][na][plane]) or NULL
 *   prev_in[3] periodic memory from the previous sweep ([nf][na][plane]);
 *              read only when have_prev != 0
 *   prev_out[3] receives this sweep's intensity on each ray's outgoing plane of
 *              every periodic axis
 *   bin_active [nf] or NULL: bins with a zero entry are skipped and their
 *              outputs left untouched
 *   J, lam [nf][cells]; H [3][nf][cells]; K [6][nf][cells] (xx yy zz xy xz yz)
 * Outputs are overwritten.  Returns 0, or -1 when scratch memory runs out.
 */
int orc_sweep(const orc_grid *g, const double *mu, const double *w,
              const double *chi, const double *B, const double *S,
              const double *const *fixed, const double *const *prev_in,
              int have_prev, double *const *prev_out, const int32_t *bin_active,
              double *J, double *H, double *K, double *lam)
{
    const int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int64_t tot = ncell * g->nf;
    for (int f = 0; f < g->nf; ++f) {
        if (bin_active && !bin_active[f]) continue;
        memset(J + f * ncell, 0, sizeof(double) * ncell);
        memset(lam + f * ncell, 0, sizeof(double) * ncell);
        if (g->want_hk) {
            for (int q = 0; q < 3; ++q) memset(H + q * tot + f * ncell, 0, sizeof(double) * ncell);
            for (int q = 0; q < 6; ++q) memset(K + q * tot + f * ncell, 0, sizeof(double) * ncell);
        }
    }
    double *Icur = (double *)malloc(sizeof(double) * ncell);
    if (!Icur) return -1;

    for (int f = 0; f < g->nf; ++f) {
        if (bin_active && !bin_active[f]) continue;
        const double *chif = chi + f * ncell;
        const double *Bf = B + f * ncell;
        const double *Sf = S + f * ncell;
        for (int ray = 0; ray < g->na; ++ray) {
            const double *m = mu + 3 * ray;
            orc_ray r;
            ray_geometry(m, g->h, &r);
            double wv[4];
            face_weights(&r, wv);

            orc_ctx c = {g, f, ray, chif, Sf, Bf, Icur, fixed, prev_in, have_prev, Sf};
            const double wk = w[ray];
            const double mx = m[0], my = m[1], mz = m[2];

            for (int64_t idx = 0; idx < ncell; ++idx) {
                int cpos[3];
                visit_position(g, &r, idx, cpos);
                double I0, ldiag;
                vertex_solve(&c, &r, wv, cpos, &I0, &ldiag);
                int64_t id = cell_index(g, cpos[0], cpos[1], cpos[2]);
                Icur[id] = I0;

                int64_t o = (int64_t)f * ncell + id;
                J[o] += wk * I0;
                lam[o] += wk * ldiag;
                if (g->want_hk) {
                    H[0 * tot + o] += wk * mx * I0;
                    H[1 * tot + o] += wk * my * I0;
                    H[2 * tot + o] += wk * mz * I0;
                    K[0 * tot + o] += wk * mx * mx * I0;
                    K[1 * tot + o] += wk * my * my * I0;
                    K[2 * tot + o] += wk * mz * mz * I0;
                    K[3 * tot + o] += wk * mx * my * I0;
                    K[4 * tot + o] += wk * mx * mz * I0;
                    K[5 * tot + o] += wk * my * mz * I0;
                }
            }
            save_periodic(g, &r, f, ray, Icur, prev_out);
        }
    }
    free(Icur);
    return 0;
}

/*
 * One Gauss-Seidel iteration of the ALI (section 3.4): the scheme the paper takes
 * from Trujillo Bueno & Fabiani Bendicho (1995) for one dimension and generalises to
 * 2D and 3D with bilinear interpolation of the upwind intensity.  The update of
 * eq. dsjacobi is applied to a vertex as soon as its J is complete, and every later
 * short characteristic sees the new S.  The ordering here takes the horizontal
 * planes as its blocks (z is the vertical, non-periodic axis):
 *
 *   1. the rays going up (direction sign +1 along z) are swept over the whole grid
 *      with the old S; no vertex has been updated yet, so their intensities are
 *      final, and their share of J is kept;
 *   2. the planes are then taken from the top (k = nz - 1) down.  Every ray going
 *      down is advanced over plane k in its row-major order (the planes above are
 *      final, plane k still holds the old S), which completes J on plane k; the
 *      plane's S is updated with eq. dsjacobi; and the plane's downward intensities
 *      are computed again from the updated S, since the planes below read them (the
 *      paper's update of the outgoing intensities).
 *
 * Every vertex of plane k is then updated with J = Lambda applied to S holding the
 * new values on the planes above and the old ones elsewhere: Gauss-Seidel with the
 * planes in descending order and Jacobi within a plane.  With first-order segments
 * and bilinear interpolation a ray going up depends only on vertices at or below its
 * own plane, so its contributions need no correction (the paper's correction of the
 * upward share with saved weights arises with the parabolic source, which reads the
 * downwind S).
 *
 * Periodic ghosts (x, y) read prev_in, the memory of the previous iteration, for the
 * whole iteration; before any iteration they take S as it was when the iteration
 * began.  prev_out receives the upward rays' outgoing planes from step 1 and the
 * downward rays' from the recomputed planes of step 2.
 *
 *   eps, B, chi [nf][cells];  S [nf][cells] in: S^n, out: S^{n+1}
 *   J   [nf][cells] out: the J each vertex was updated with
 *   lam [nf][cells] out: Lambda* = sum_k w_k psi0_k
 *   dS  [nf][cells] out: the update of eq. dsjacobi
 * Needs order = 0, interp = 0 and a non-periodic z axis.  Bins with bin_active[f] = 0
 * are skipped.  Returns 0, -1 when scratch memory runs out, -2 for an unsupported grid.
 */
int orc_gs_iteration(const orc_grid *g, const double *mu, const double *w,
                     const double *chi, const double *B, const double *eps, double *S,
                     const double *const *fixed, const double *const *prev_in, int have_prev,
                     double *const *prev_out, const int32_t *bin_active,
                     double *J, double *lam, double *dS)
{
    if (g->order != 0 || g->interp != 0 || is_periodic(g, 2)) return -2;
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int64_t nxy = (int64_t)nx * ny;
    int ndown = 0;
    for (int ray = 0; ray < g->na; ++ray) ndown += mu[3 * ray + 2] < 0.0;
    double *Iup = (double *)malloc(sizeof(double) * ncell);
    double *Idn = (double *)malloc(sizeof(double) * ncell * (ndown > 0 ? ndown : 1));
    double *S0 = (double *)malloc(sizeof(double) * ncell);
    if (!Iup || !Idn || !S0) {
        free(Iup);
        free(Idn);
        free(S0);
        return -1;
    }

    for (int f = 0; f < g->nf; ++f) {
        if (bin_active && !bin_active[f]) continue;
        const double *chif = chi + f * ncell;
        const double *Bf = B + f * ncell;
        const double *ef = eps + f * ncell;
        double *Sf = S + f * ncell;
        double *Jf = J + f * ncell;
        double *lf = lam + f * ncell;
        double *dSf = dS + f * ncell;
        memcpy(S0, Sf, sizeof(double) * ncell);
        memset(Jf, 0, sizeof(double) * ncell);
        memset(lf, 0, sizeof(double) * ncell);

        /* 1. rays going up, the whole grid with the old S */
        for (int ray = 0; ray < g->na; ++ray) {
            const double *m = mu + 3 * ray;
            if (m[2] < 0.0) continue;
            orc_ray r;
            ray_geometry(m, g->h, &r);
            double wv[4];
            face_weights(&r, wv);
            orc_ctx c = {g, f, ray, chif, Sf, Bf, Iup, fixed, prev_in, have_prev, S0};
            for (int64_t idx = 0; idx < ncell; ++idx) {
                int cpos[3];
                visit_position(g, &r, idx, cpos);
                double I0, ld;
                vertex_solve(&c, &r, wv, cpos, &I0, &ld);
                const int64_t id = cell_index(g, cpos[0], cpos[1], cpos[2]);
                Iup[id] = I0;
                Jf[id] += w[ray] * I0;
                lf[id] += w[ray] * ld;
            }
            save_periodic(g, &r, f, ray, Iup, prev_out);
        }

        /* 2. planes from the top down: the downward rays over plane k with the current
           S, the update of plane k, the plane's downward intensities again */
        for (int kk = 0; kk < nz; ++kk) {
            const int k = nz - 1 - kk;
            for (int pass = 0; pass < 2; ++pass) {
                int slot = 0;
                for (int ray = 0; ray < g->na; ++ray) {
                    const double *m = mu + 3 * ray;
                    if (m[2] >= 0.0) continue;
                    double *Ir = Idn + (int64_t)slot * ncell;
                    ++slot;
                    orc_ray r;
                    ray_geometry(m, g->h, &r);
                    double wv[4];
                    face_weights(&r, wv);
                    orc_ctx c = {g, f, ray, chif, Sf, Bf, Ir, fixed, prev_in, have_prev, S0};
                    for (int64_t p = 0; p < nxy; ++p) {
                        const int ox = (int)(p % nx), oy = (int)(p / nx);
                        int cpos[3];
                        cpos[0] = (r.sgn[0] > 0) ? ox : nx - 1 - ox;
                        cpos[1] = (r.sgn[1] > 0) ? oy : ny - 1 - oy;
                        cpos[2] = k;
                        double I0, ld;
                        vertex_solve(&c, &r, wv, cpos, &I0, &ld);
                        const int64_t id = cell_index(g, cpos[0], cpos[1], cpos[2]);
                        Ir[id] = I0;
                        if (pass == 0) {
                            Jf[id] += w[ray] * I0;
                            lf[id] += w[ray] * ld;
                        }
                    }
                }
                if (pass == 1) break;
                for (int64_t p = 0; p < nxy; ++p) {
                    const int64_t id = (int64_t)k * nxy + p;
                    const double e = ef[id];
                    const double d = ((1.0 - e) * Jf[id] + e * Bf[id] - Sf[id]) / (1.0 - (1.0 - e) * lf[id]);
                    dSf[id] = d;
                    Sf[id] = Sf[id] + d;
                }
            }
        }
        int slot = 0;
        for (int ray = 0; ray < g->na; ++ray) {
            const double *m = mu + 3 * ray;
            if (m[2] >= 0.0) continue;
            orc_ray r;
            ray_geometry(m, g->h, &r);
            save_periodic(g, &r, f, ray, Idn + (int64_t)slot * ncell, prev_out);
            ++slot;
        }
    }
    free(Iup);
    free(Idn);
    free(S0);
    return 0;
}

/*
 * One Gauss-Seidel iteration in the zone order of section 3.4 (Fig. f:sweep): the
 * sweep advances with i the fastest index, then j, then k; the backward sweep runs
 * it in reverse, so the zones are updated one at a time from the top corner
 * (nx-1, ny-1, nz-1) down to (0, 0, 0): planes from the top, rows from the back,
 * i descending.  When a zone is updated, every intensity it sums has been computed
 * with the current S: the new S of every zone updated before it in this iteration
 * and the old S elsewhere.  This is what the paper's corrections with saved weights
 * and its update of the outgoing intensities achieve once they are carried through
 * completely; written out here without them, as the definition of the iteration:
 *
 *     for each zone z in the order above:
 *         J_z = sum_k w_k I_k(z)   with I_k from the current S
 *         S_z += ((1 - eps) J_z + eps B - S_z) / (1 - (1 - eps) Lambda*_z)   (eq. dsjacobi)
 *
 * Evaluation.  The intensities on plane k depend only on plane k itself, on the
 * plane upwind along z and on S; when plane k is being updated, the planes above are
 * final (their zones are all updated) and the planes below still hold the old S.  So
 * the rays going up are swept once over the whole grid with the old S (their values
 * below plane k stay exact while plane k is updated); the rays going down are swept
 * over plane k once the plane above is final; and before each zone of plane k is
 * updated every ray's intensities on plane k are computed again from the current S
 * (each ray in its own row-major order inside the plane).  After the last zone of the
 * plane the downward intensities on plane k are computed once more with its final S,
 * for the plane below.  This costs n_rays * nx * ny vertex solutions per zone: the
 * oracle is for small grids.
 *
 * Ghost vertices follow the rules of the formal solution: chi and S of the folded
 * vertex (current values), intensity from the boundary condition, or on periodic
 * axes the memory of the previous iteration (before any iteration: S of the wrapped
 * vertex as the iteration began).  prev_out receives the rays going up from the
 * sweep with the old S and the rays going down from their final planes.
 *
 * Arguments and layouts as orc_gs_iteration.  Needs order = 0, interp = 0 and a
 * non-periodic z axis.  Returns 0, -1 when scratch memory runs out, -2 for an
 * unsupported grid.
 */
int orc_gs_point_iteration(const orc_grid *g, const double *mu, const double *w,
                           const double *chi, const double *B, const double *eps, double *S,
                           const double *const *fixed, const double *const *prev_in, int have_prev,
                           double *const *prev_out, const int32_t *bin_active,
                           double *J, double *lam, double *dS)
{
    if (g->order != 0 || g->interp != 0 || is_periodic(g, 2)) return -2;
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int64_t nxy = (int64_t)nx * ny;
    double *I = (double *)malloc(sizeof(double) * ncell * (g->na > 0 ? g->na : 1));
    double *S0 = (double *)malloc(sizeof(double) * ncell);
    if (!I || !S0) {
        free(I);
        free(S0);
        return -1;
    }

    for (int f = 0; f < g->nf; ++f) {
        if (bin_active && !bin_active[f]) continue;
        const double *chif = chi + f * ncell;
        const double *Bf = B + f * ncell;
        const double *ef = eps + f * ncell;
        double *Sf = S + f * ncell;
        double *Jf = J + f * ncell;
        double *lf = lam + f * ncell;
        double *dSf = dS + f * ncell;
        memcpy(S0, Sf, sizeof(double) * ncell);

        /* the rays going up over the whole grid with the old S */
        for (int ray = 0; ray < g->na; ++ray) {
            const double *m = mu + 3 * ray;
            if (m[2] < 0.0) continue;
            orc_ray r;
            ray_geometry(m, g->h, &r);
            double wv[4];
            face_weights(&r, wv);
            double *Ir = I + (int64_t)ray * ncell;
            orc_ctx c = {g, f, ray, chif, Sf, Bf, Ir, fixed, prev_in, have_prev, S0};
            for (int64_t idx = 0; idx < ncell; ++idx) {
                int cpos[3];
                visit_position(g, &r, idx, cpos);
                double I0, ld;
                vertex_solve(&c, &r, wv, cpos, &I0, &ld);
                Ir[cell_index(g, cpos[0], cpos[1], cpos[2])] = I0;
            }
            save_periodic(g, &r, f, ray, Ir, prev_out);
        }

        for (int kk = 0; kk < nz; ++kk) {
            const int k = nz - 1 - kk;
            /* zones of plane k in the backward order; last pass: the final plane */
            for (int64_t zz = 0; zz <= nxy; ++zz) {
                const int last = zz == nxy;
                const int zi = last ? 0 : nx - 1 - (int)(zz % nx);
                const int zj = last ? 0 : ny - 1 - (int)(zz / nx);
                const int64_t zid = cell_index(g, zi, zj, k);
                double Jz = 0.0, lz = 0.0;
                for (int ray = 0; ray < g->na; ++ray) {
                    const double *m = mu + 3 * ray;
                    if (last && m[2] >= 0.0) continue;
                    orc_ray r;
                    ray_geometry(m, g->h, &r);
                    double wv[4];
                    face_weights(&r, wv);
                    double *Ir = I + (int64_t)ray * ncell;
                    orc_ctx c = {g, f, ray, chif, Sf, Bf, Ir, fixed, prev_in, have_prev, S0};
                    /* the ray's intensities on plane k from the current S, row-major
                       from its upwind corner inside the plane */
                    for (int64_t p = 0; p < nxy; ++p) {
                        const int ox = (int)(p % nx), oy = (int)(p / nx);
                        int cpos[3];
                        cpos[0] = (r.sgn[0] > 0) ? ox : nx - 1 - ox;
                        cpos[1] = (r.sgn[1] > 0) ? oy : ny - 1 - oy;
                        cpos[2] = k;
                        double I0, ld;
                        vertex_solve(&c, &r, wv, cpos, &I0, &ld);
                        const int64_t id = cell_index(g, cpos[0], cpos[1], cpos[2]);
                        Ir[id] = I0;
                        if (id == zid) {
                            Jz += w[ray] * I0;
                            lz += w[ray] * ld;
                        }
                    }
                }
                if (last) break;
                const double e = ef[zid];
                const double d = ((1.0 - e) * Jz + e * Bf[zid] - Sf[zid]) / (1.0 - (1.0 - e) * lz);
                Jf[zid] = Jz;
                lf[zid] = lz;
                dSf[zid] = d;
                Sf[zid] = Sf[zid] + d;
            }
        }
        for (int ray = 0; ray < g->na; ++ray) {
            const double *m = mu + 3 * ray;
            if (m[2] >= 0.0) continue;
            orc_ray r;
            ray_geometry(m, g->h, &r);
            save_periodic(g, &r, f, ray, I + (int64_t)ray * ncell, prev_out);
        }
    }
    free(I);
    free(S0);
    return 0;
}

/* Geometry of one ray, exported for tests: d, a, b, signs; s, fa, fb. */
void orc_ray_info(const double mu[3], const double h[3], int32_t *iout, double *dout)
{
    orc_ray r;
    ray_geometry(mu, h, &r);
    iout[0] = r.d;
    iout[1] = r.a;
    iout[2] = r.b;
    iout[3] = r.sgn[0];
    iout[4] = r.sgn[1];
    iout[5] = r.sgn[2];
    dout[0] = r.s;
    dout[1] = r.fa;
    dout[2] = r.fb;
}
