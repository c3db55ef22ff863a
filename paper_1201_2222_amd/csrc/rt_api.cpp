// Host runtime and C ABI of librtsc (declarations in include/rt.h).
//
// Owns the per-problem device state, the angle set and per-ray geometry, the
// tile schedule of the wavefront sweep, and the Jacobi ALI driver.  Every step of
// the formal solution and of the iteration runs in the HIP kernels of
// rt_kernels.hip; this file only validates, allocates and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <utility>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/rt.h"
#include "rt_internal.h"

using namespace rtsc;

// A device and the last error of the calls made through it (rt_context_create).
struct rt_context {
    int device = 0;
    std::mutex mu;
    std::string err;
};

namespace {

thread_local std::string g_err;
thread_local rt_context *t_ctx = nullptr;   // context of the call in progress on this thread

rt_status fail(rt_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    if (t_ctx) {
        std::lock_guard<std::mutex> lk(t_ctx->mu);
        t_ctx->err = buf;
    }
    return s;
}

// For the duration of one entry point: failures are recorded in `ctx` too, and the
// device of the problem (or context) is current; the caller's context and device
// are restored on return.
class CallScope {
  public:
    CallScope(rt_context *ctx, int device) : prev_ctx_(t_ctx)
    {
        t_ctx = ctx;
        int cur = -1;
        if (device >= 0 && hipGetDevice(&cur) == hipSuccess && cur != device && hipSetDevice(device) == hipSuccess) {
            prev_dev_ = cur;
        }
        (void)hipGetLastError();
    }
    ~CallScope()
    {
        if (prev_dev_ >= 0) (void)hipSetDevice(prev_dev_);
        t_ctx = prev_ctx_;
    }
    CallScope(const CallScope &) = delete;
    CallScope &operator=(const CallScope &) = delete;

  private:
    rt_context *prev_ctx_;
    int prev_dev_ = -1;
};

#define HIP_TRY(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(RT_E_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                              \
    } while (0)

// ---------------------------------------------------------------------------------
// Level-symmetric angle set (section 3.2).  Per octant: directions (mu_i, mu_j, mu_k)
// with i + j + k = m + 2 (m = n_mu/2), levels mu_i^2 = a + (i-1) 2(1-3a)/(n_mu-2), one
// weight per permutation class.  Given a = mu_1^2 the class weights follow linearly
// from the conditions <mu_x^2p> = 1/(2p+1), p = 0, 2..m-1; a itself is the smallest
// root in (0, 1/3) of the remaining condition p = m with all weights positive.
// Evaluated in long double; the root by bracketing and bisection.
// ---------------------------------------------------------------------------------
struct LsClass {
    int i, j, k;
};

std::vector<LsClass> ls_classes(int m)
{
    std::vector<LsClass> c;
    for (int i = 1; i <= m; ++i)
        for (int j = i; j <= m; ++j)
            for (int k = j; k <= m; ++k)
                if (i + j + k == m + 2) c.push_back({i, j, k});
    return c;
}

// sum over the distinct permutations of a class of (level of the first index)^p
long double class_moment(const LsClass &c, int p, const std::vector<long double> &lev)
{
    int t[3] = {c.i, c.j, c.k};
    std::sort(t, t + 3);
    long double acc = 0.0L;
    do {
        acc += std::pow(lev[t[0] - 1], (long double)p);
    } while (std::next_permutation(t, t + 3));
    return acc;
}

bool ls_weights(int n_mu, long double a, std::vector<long double> &wc, long double &resid)
{
    const int m = n_mu / 2;
    std::vector<LsClass> cls = ls_classes(m);
    const int nc = (int)cls.size();
    std::vector<long double> lev(m);
    const long double step = 2.0L * (1.0L - 3.0L * a) / (n_mu - 2);
    for (int i = 0; i < m; ++i) lev[i] = a + i * step;
    std::vector<int> ps;
    ps.push_back(0);
    for (int p = 2; p < m; ++p) ps.push_back(p);
    // augmented system, Gaussian elimination with partial pivoting
    std::vector<std::vector<long double>> M(nc, std::vector<long double>(nc + 1));
    for (int r = 0; r < nc; ++r) {
        for (int c = 0; c < nc; ++c) M[r][c] = class_moment(cls[c], ps[r], lev);
        M[r][nc] = 1.0L / (2 * ps[r] + 1);
    }
    for (int c = 0; c < nc; ++c) {
        int piv = c;
        for (int r = c + 1; r < nc; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (std::fabs(M[piv][c]) < 1e-300L) return false;
        std::swap(M[c], M[piv]);
        for (int r = 0; r < nc; ++r) {
            if (r == c) continue;
            const long double f = M[r][c] / M[c][c];
            for (int k = c; k <= nc; ++k) M[r][k] -= f * M[c][k];
        }
    }
    wc.assign(nc, 0.0L);
    for (int c = 0; c < nc; ++c) wc[c] = M[c][nc] / M[c][c];
    resid = -1.0L / (2 * m + 1);
    for (int c = 0; c < nc; ++c) resid += wc[c] * class_moment(cls[c], m, lev);
    return true;
}

bool level_symmetric(int n_mu, std::vector<double> &mu, std::vector<double> &w)
{
    const int m = n_mu / 2;
    long double a;
    std::vector<long double> wc;
    if (n_mu == 2) {
        a = 1.0L / 3.0L;
        wc.assign(1, 1.0L);
    } else {
        const int N = 4000;
        const long double lo = 1e-6L, hi = 1.0L / 3.0L - 1e-6L;
        bool found = false;
        long double r0 = 0.0L;
        std::vector<long double> wtmp;
        bool ok0 = ls_weights(n_mu, lo, wtmp, r0);
        long double x0 = lo;
        for (int s = 1; s <= N && !found; ++s) {
            const long double x1 = lo + (hi - lo) * s / N;
            long double r1;
            const bool ok1 = ls_weights(n_mu, x1, wtmp, r1);
            if (ok0 && ok1 && (r0 == 0.0L || (r0 < 0.0L) != (r1 < 0.0L))) {
                long double xa = x0, xb = x1, ra = r0;
                for (int it = 0; it < 200; ++it) {
                    const long double xm = 0.5L * (xa + xb);
                    long double rm;
                    ls_weights(n_mu, xm, wtmp, rm);
                    if (rm == 0.0L || xm == xa || xm == xb) {
                        xa = xb = xm;
                        break;
                    }
                    if ((rm < 0.0L) == (ra < 0.0L)) {
                        xa = xm;
                        ra = rm;
                    } else {
                        xb = xm;
                    }
                }
                const long double root = 0.5L * (xa + xb);
                long double rr;
                if (ls_weights(n_mu, root, wc, rr) &&
                    std::all_of(wc.begin(), wc.end(), [](long double v) { return v > 0.0L; })) {
                    a = root;
                    found = true;
                }
            }
            x0 = x1;
            r0 = r1;
            ok0 = ok1;
        }
        if (!found) return false;
    }
    std::vector<long double> lev(m);
    for (int i = 0; i < m; ++i) lev[i] = (n_mu == 2) ? a : a + i * 2.0L * (1.0L - 3.0L * a) / (n_mu - 2);
    std::vector<LsClass> cls = (n_mu == 2) ? std::vector<LsClass>{{1, 1, 1}} : ls_classes(m);
    // directions of one octant in lexicographic order of (i, j, k), with their class weight
    std::vector<double> mo, wo;
    for (int i = 1; i <= m; ++i)
        for (int j = 1; j <= m; ++j)
            for (int k = 1; k <= m; ++k) {
                if (i + j + k != m + 2) continue;
                int t[3] = {i, j, k};
                std::sort(t, t + 3);
                int ci = -1;
                for (size_t c = 0; c < cls.size(); ++c)
                    if (cls[c].i == t[0] && cls[c].j == t[1] && cls[c].k == t[2]) ci = (int)c;
                mo.push_back((double)std::sqrt(lev[i - 1]));
                mo.push_back((double)std::sqrt(lev[j - 1]));
                mo.push_back((double)std::sqrt(lev[k - 1]));
                wo.push_back((double)(wc[ci] / 8.0L));
            }
    const int per = (int)wo.size();
    mu.assign((size_t)8 * per * 3, 0.0);
    w.assign((size_t)8 * per, 0.0);
    for (int o = 0; o < 8; ++o)
        for (int r = 0; r < per; ++r) {
            for (int q = 0; q < 3; ++q) mu[((size_t)o * per + r) * 3 + q] = ((o >> q) & 1 ? -1.0 : 1.0) * mo[r * 3 + q];
            w[(size_t)o * per + r] = wo[r];
        }
    return true;
}

int octant_of(const double *m) { return (m[0] < 0.0 ? 1 : 0) | (m[1] < 0.0 ? 2 : 0) | (m[2] < 0.0 ? 4 : 0); }

// Short-characteristic geometry of a ray on a uniform grid (section 3.3): the face
// plane crossed first going upwind, path length and bilinear face weights.
RayGeo ray_geometry(const double m[3], const double h[3], double wk, int gidx)
{
    RayGeo g{};
    double len[3];
    for (int q = 0; q < 3; ++q) len[q] = (m[q] == 0.0) ? std::numeric_limits<double>::infinity() : h[q] / std::fabs(m[q]);
    int d = 2;  // equal lengths: z before y before x
    if (len[1] < len[d]) d = 1;
    if (len[0] < len[d]) d = 0;
    g.d = d;
    g.a = (d == 0) ? 1 : 0;
    g.b = (d == 2) ? 1 : 2;
    g.oct = octant_of(m);
    g.gidx = gidx;
    g.s = len[d];
    const double fa = std::min(1.0, g.s * std::fabs(m[g.a]) / h[g.a]);
    const double fb = std::min(1.0, g.s * std::fabs(m[g.b]) / h[g.b]);
    g.w4[0] = (1.0 - fa) * (1.0 - fb);
    g.w4[1] = fa * (1.0 - fb);
    g.w4[2] = (1.0 - fa) * fb;
    g.w4[3] = fa * fb;
    g.fa = fa;
    g.fb = fb;
    g.wk = wk;
    for (int q = 0; q < 3; ++q) g.mu[q] = m[q];
    return g;
}

}  // namespace

struct rt_problem {
    rt_problem_desc desc{};
    rt_context *ctx = nullptr;         // context it was created in, or null
    int device = 0;                    // HIP device holding its state
    std::atomic<int> server_refs{0};   // queued or running server requests on it
    // caller arrays in FP32 (desc.in_dtype): FP64 copies of the caller's S and J that
    // the solvers work on, and FP64 staging of the moments outputs (made on first use)
    bool usr32 = false;
    double *stS = nullptr, *stJ = nullptr;
    double *mst[8]{};
    int n[3]{};
    int nf = 0, na = 0, R = 0;
    int nt[3]{};
    int nstages = 0;
    int64_t cells = 0;
    int64_t plane[3]{};
    int64_t pplane[3]{};               // values per face-plane slot (FacePlane::slot)
    int periodic[3]{};
    bool f32 = false;
    bool cold = true;
    bool have_fields = false;
    std::vector<RayGeo> rays;          // octant-major
    std::vector<double> w_nu;
    std::vector<int> stage_off;        // [nstages + 1]
    // device state
    RayGeo *d_rays = nullptr;
    int *d_tiles = nullptr;
    int *d_stage_tab = nullptr;        // device copy of stage_off (batched launches)
    double *chi64 = nullptr, *eps = nullptr, *B = nullptr, *lam = nullptr;
    float *chi32 = nullptr;
    void *face[3]{};                   // Real [nf][na][nt_q][pplane_q]
    double *wrap[3]{};                 // [nf][na][2][plane_q] on periodic axes
    void *part = nullptr;              // Real [npart][nf][cells]
    int npart = 8;                     // partial-sum slots: 8 octants, or kPlaneParts (plane order)
    // plane-ordered sweep (quadratic upwind intensity)
    bool plane_order = false;
    void *planes = nullptr;            // Real [nf][na][2][pmax]
    double *wrapI = nullptr;           // [nf][na][pmax] (difference form)
    int64_t pmax = 0;
    int *d_cls_off = nullptr;          // [kPlaneParts + 1]
    int *d_cls_rays = nullptr;         // [na]
    int plane_tiles_a[3]{}, plane_ntiles[3]{};
    int *frozen = nullptr, *parity = nullptr, *iters = nullptr, *flags = nullptr;
    double *resid = nullptr;
    unsigned long long *blockmax = nullptr;  // [nf][kUpdateBlocks]
    int waves = 1;                     // waves per sweep workgroup
    size_t lds_limit = 65536;          // LDS bytes a workgroup may use on the device
    bool persistent = false;           // one launch per sweep (dependency flags)
    int ntiles = 0;                    // tiles per (bin, octant)
    int bpo = 1;                       // persistent workgroups per octant
    uint64_t wait_ticks = 0;           // bound of one dependency wait in device wall-clock ticks
    int wall_khz = 100000;             // the device's constant-rate clock
    int *dag_counter = nullptr;        // [8] ticket counters
    // moments epilogue scratch (allocated on first use)
    int mom_nfc = 0;                   // bins per moments chunk
    void *mom_part = nullptr;          // Real [8][10][mom_nfc][cells]
    double *mom_tmp = nullptr;         // [10][mom_nfc][cells]
    double *mom_q = nullptr;           // [mom_nfc][cells]
    double *mom_qint = nullptr;        // [cells] when the caller does not ask for Q_int
    double *mom_wnu = nullptr;         // [nf]
    double *mom_sum = nullptr;         // [1024 + 1]
    double *h_sum = nullptr;           // pinned scalar
    int *dag_done = nullptr;           // [nf][8][ntiles] completion epochs
    // Gauss-Seidel ALI (allocated on first use)
    void *gs_planes = nullptr;         // Real [nf][nd][2][nx ny]
    void *gs_part = nullptr;           // Real [nd][nf][nx ny]
    void *gs_coef = nullptr;           // Real [nf][ns][4][nx ny]
    void *gs_gh = nullptr;             // Real [nf][ns][4][max(nx, ny)]
    double *gs_ghS = nullptr;          // [nf][ns][2][max(nx, ny)]
    void *gs_chi_t = nullptr;          // Real [nf][nz][nx][ny]
    double *gs_S_t = nullptr;          // [nf][nz][nx][ny]
    int *d_gs_down = nullptr;          // [nd] rays going down, shallow ones first
    // timing of the Gauss-Seidel chain launches (one iteration per check interval)
    std::vector<hipEvent_t> gs_ev;     // [2 nz]: before and after the chain launch of step t
    bool gs_prof_pending = false;
    double gs_prof_ms = 0.0, gs_prof_updates = 0.0, gs_pending_updates = 0.0;
    int64_t gs_prof_launches = 0;
    int gs_nd = 0, gs_ns = 0;
    int *h_flags = nullptr;            // pinned host copy of flags
    int *h_frozen = nullptr;           // pinned host copy of frozen
    std::vector<void *> allocs;
    // ALI chunks captured as graphs (rt_problem_use_graphs); at most two cached: the
    // full chunk and the last, shorter one
    struct GraphEntry {
        int k = 0;
        bool gs = false;
        const double *S = nullptr, *J = nullptr;
        double delta_c = 0.0;
        int per_bin_stop = 0, fixed = 0;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;  // capture stream (non-blocking, default priority)
    std::vector<GraphEntry> graphs;
    // sweep-kernel timing (rt_problem_profile)
    bool prof = false;
    bool prof_pending = false;
    std::vector<hipEvent_t> ev;        // start/stop of a timed sweep
    double prof_ms = 0.0, prof_updates = 0.0, prof_pending_updates = 0.0;
    int64_t prof_launches = 0, prof_sweeps = 0;
};

namespace {

size_t real_size(const rt_problem_desc *d) { return d->precision == RT_F32 ? sizeof(float) : sizeof(double); }

rt_status validate(const rt_problem_desc *d, int *na_out)
{
    if (!d) return fail(RT_E_INVALID, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(RT_E_INVALID, "grid dimensions must be >= 1");
    if (d->nx > 8000 || d->ny > 8000 || d->nz > 8000) return fail(RT_E_INVALID, "grid dimension above 8000");
    if (d->nf < 1 || d->nf > 65535) return fail(RT_E_INVALID, "nf must be in [1, 65535]");
    if ((int64_t)d->nx * d->ny * d->nz > INT32_MAX)
        return fail(RT_E_UNSUPPORTED, "more than 2^31 - 1 vertices per bin (the sweep indexes a bin with 32 bits)");
    if (!(d->dx > 0.0) || !(d->dy > 0.0) || !(d->dz > 0.0) || !std::isfinite(d->dx) || !std::isfinite(d->dy) ||
        !std::isfinite(d->dz))
        return fail(RT_E_INVALID, "dx, dy, dz must be finite and > 0");
    if (d->precision != RT_F64 && d->precision != RT_F32) return fail(RT_E_INVALID, "unknown precision");
    if (d->in_dtype != RT_DTYPE_F64 && d->in_dtype != RT_DTYPE_F32) return fail(RT_E_INVALID, "unknown in_dtype");
    if (d->tile != 0 && d->tile != kTile) return fail(RT_E_UNSUPPORTED, "tile edge %d not built (only %d)", d->tile, kTile);
    if (d->schedule < RT_SCHED_DEFAULT || d->schedule > RT_SCHED_PERSISTENT) return fail(RT_E_INVALID, "unknown schedule");
    if (d->order != RT_SC_LINEAR && d->order != RT_SC_BEZIER) return fail(RT_E_INVALID, "unknown order");
    if (d->interp != RT_INTERP_BILINEAR && d->interp != RT_INTERP_QUADRATIC)
        return fail(RT_E_INVALID, "unknown upwind interpolation");
    if (d->interp == RT_INTERP_QUADRATIC && d->order != RT_SC_LINEAR)
        return fail(RT_E_UNSUPPORTED, "the quadratic upwind intensity is built with first-order segments only");
    if (d->schedule == RT_SCHED_PERSISTENT && (d->order != RT_SC_LINEAR || d->interp != RT_INTERP_BILINEAR))
        return fail(RT_E_UNSUPPORTED, "the persistent schedule is built for first-order segments with bilinear upwind values");
    for (int q = 0; q < 3; ++q) {
        for (int k : {d->bc_lo[q], d->bc_hi[q]})
            if (k < RT_BC_VACUUM || k > RT_BC_FIXED) return fail(RT_E_INVALID, "unknown boundary kind on axis %d", q);
        if ((d->bc_lo[q] == RT_BC_PERIODIC) != (d->bc_hi[q] == RT_BC_PERIODIC))
            return fail(RT_E_INVALID, "axis %d periodic on one face only", q);
        if (d->bc_lo[q] == RT_BC_FIXED && !d->I_fixed[2 * q]) return fail(RT_E_INVALID, "FIXED low face %d without data", q);
        if (d->bc_hi[q] == RT_BC_FIXED && !d->I_fixed[2 * q + 1]) return fail(RT_E_INVALID, "FIXED high face %d without data", q);
    }
    int na;
    if (d->mu) {
        if (!d->w) return fail(RT_E_INVALID, "mu given without w");
        na = d->na;
        if (na < 8 || na % 8 != 0 || na > 8 * 64) return fail(RT_E_INVALID, "na must be a multiple of 8 in [8, 512]");
        int cnt[8] = {0};
        double wsum = 0.0;
        for (int k = 0; k < na; ++k) {
            const double *m = d->mu + 3 * k;
            const double nrm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
            if (!(std::fabs(nrm - 1.0) < 1e-12)) return fail(RT_E_INVALID, "ray %d is not a unit vector", k);
            if (!(d->w[k] >= 0.0)) return fail(RT_E_INVALID, "ray %d has a negative weight", k);
            ++cnt[octant_of(m)];
            wsum += d->w[k];
        }
        for (int o = 0; o < 8; ++o)
            if (cnt[o] != na / 8) return fail(RT_E_INVALID, "every octant needs na/8 rays (octant %d has %d)", o, cnt[o]);
        if (!(std::fabs(wsum - 1.0) < 1e-12)) return fail(RT_E_INVALID, "ray weights sum to %.17g, not 1", wsum);
    } else {
        if (d->n_mu != 2 && d->n_mu != 4 && d->n_mu != 6 && d->n_mu != 8 && d->n_mu != 10 && d->n_mu != 12)
            return fail(RT_E_INVALID, "n_mu must be 2, 4, 6, 8, 10 or 12");
        na = d->n_mu * (d->n_mu + 2);
    }
    if (d->w_nu)
        for (int f = 0; f < d->nf; ++f)
            if (!std::isfinite(d->w_nu[f])) return fail(RT_E_INVALID, "w_nu[%d] is not finite", f);
    *na_out = na;
    return RT_OK;
}

void tile_counts(const rt_problem_desc *d, int nt[3])
{
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int q = 0; q < 3; ++q) nt[q] = (n[q] + kTile - 1) / kTile;
}

size_t state_bytes(const rt_problem_desc *d, int na)
{
    const int64_t cells = (int64_t)d->nx * d->ny * d->nz;
    const int64_t nc = cells * d->nf;
    const size_t rs = real_size(d);
    int nt[3];
    tile_counts(d, nt);
    const int64_t plane[3] = {(int64_t)d->ny * d->nz, (int64_t)d->nx * d->nz, (int64_t)d->nx * d->ny};
    const int64_t pplane[3] = {FacePlane(d->ny, d->nz).slot(), FacePlane(d->nx, d->nz).slot(),
                               FacePlane(d->nx, d->ny).slot()};
    const int bc_per[3] = {d->bc_lo[0] == RT_BC_PERIODIC, d->bc_lo[1] == RT_BC_PERIODIC, d->bc_lo[2] == RT_BC_PERIODIC};
    size_t b = 0;
    b += (size_t)nc * 8 * 4;                       // chi64, eps, B, lam
    if (d->precision == RT_F32) b += (size_t)nc * 4;  // chi32
    if (d->interp == RT_INTERP_QUADRATIC) {
        const int64_t pmax = std::max(plane[0], std::max(plane[1], plane[2]));
        b += (size_t)d->nf * na * 2 * pmax * rs;   // two planes per ray
        if (d->precision == RT_F32) b += (size_t)d->nf * na * pmax * 8;   // FP64 last planes
        b += (size_t)kPlaneParts * nc * rs;        // partials per octant and first-crossed axis
        b += (size_t)(kPlaneParts + 1 + na) * 4;
    } else {
        for (int q = 0; q < 3; ++q) {
            b += (size_t)d->nf * na * nt[q] * pplane[q] * rs;           // face planes
            if (bc_per[q]) b += (size_t)d->nf * na * 2 * plane[q] * 8;  // periodic memory
        }
        b += (size_t)8 * nc * rs;                  // partials
    }
    if (d->in_dtype == RT_DTYPE_F32) b += (size_t)nc * 8 * 2;   // FP64 copies of the caller's S and J
    b += (size_t)d->nf * kUpdateBlocks * 8;        // residual block maxima
    b += (size_t)d->nf * 8 * nt[0] * nt[1] * nt[2] * 4 + 64;  // persistent-sweep flags
    b += (size_t)na * sizeof(RayGeo) + (size_t)nt[0] * nt[1] * nt[2] * 4 + (size_t)d->nf * 32 + 64;
    return b;
}

template <typename T>
rt_status dalloc(rt_problem *p, T **ptr, size_t count)
{
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, std::max<size_t>(count * sizeof(T), 16));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RT_E_OOM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    p->allocs.push_back(v);
    *ptr = static_cast<T *>(v);
    return RT_OK;
}

template <typename Real>
SweepArgs<Real> sweep_args(rt_problem *p, const double *S)
{
    SweepArgs<Real> A{};
    for (int q = 0; q < 3; ++q) {
        A.n[q] = p->n[q];
        A.nt[q] = p->nt[q];
        A.bc_lo[q] = p->desc.bc_lo[q];
        A.bc_hi[q] = p->desc.bc_hi[q];
        A.periodic[q] = p->periodic[q];
        A.plane[q] = p->plane[q];
        A.pplane[q] = p->pplane[q];
        A.face[q] = static_cast<Real *>(p->face[q]);
        A.wrap[q] = p->wrap[q];
    }
    A.nf = p->nf;
    A.na = p->na;
    A.R = p->R;
    A.cells = p->cells;
    A.rays = p->d_rays;
    A.chi = p->f32 ? reinterpret_cast<const Real *>(p->chi32) : reinterpret_cast<const Real *>(p->chi64);
    A.S = S;
    A.B = p->B;
    for (int k = 0; k < 6; ++k) A.fixed[k] = p->desc.I_fixed[k];
    A.part = static_cast<Real *>(p->part);
    A.f0 = 0;
    A.nfc = p->nf;
    A.tiles = p->d_tiles;
    A.frozen = p->frozen;
    A.parity = p->parity;
    A.stage_tab = p->d_stage_tab;
    A.nstages = p->nstages;
    A.order = p->desc.order;
    A.noct = 8;
    return A;
}

// Waves per sweep workgroup: one per ray of the octant, capped so the dynamic LDS
// (chi and S tiles; a cube of I and a partial-sum tile per wave) fits
// the device's per-workgroup limit.
// Workgroups per octant of the persistent sweep: as many as fit on the device at the
// problem's wave count, at most one per tile and bin.
void persistent_grid(rt_problem *p)
{
    int dev = 0, per_cu = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        persistent_blocks_per_cu(p->f32 ? 4 : 8, p->waves, &per_cu) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 8) ncu = 8;
    (void)hipGetLastError();
    p->bpo = std::max(1, std::min(per_cu * ncu / 8, p->ntiles * p->nf));
}

int sweep_waves(int R, bool f32, int order, size_t lds_limit)
{
    int w = std::min(R, kMaxWaves);
    while (w > 1 && sweep_lds_bytes(f32 ? 4 : 8, w, 1, R > w, order) > lds_limit) --w;
    return w;
}

// One formal solution over every active bin: the tile stages in order.
// Accumulate the duration of a timed sweep once its events have completed: two
// events bracket the back-to-back stage launches (per-launch events would delay
// every launch), so a launch's share includes the gap to the next launch.
rt_status collect_timing(rt_problem *p)
{
    if (p->gs_prof_pending) {
        // chain launches of steps 1 .. nz-1 (those that compute a plane and recompute
        // the one above: one kernel variant)
        const int nz = p->n[2];
        HIP_TRY(hipEventSynchronize(p->gs_ev[2 * (nz - 1) + 1]));
        for (int t = 1; t < nz; ++t) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, p->gs_ev[2 * t], p->gs_ev[2 * t + 1]));
            p->gs_prof_ms += ms;
        }
        p->gs_prof_launches += nz - 1;
        p->gs_prof_updates += p->gs_pending_updates;
        p->gs_prof_pending = false;
    }
    if (!p->prof_pending) return RT_OK;
    HIP_TRY(hipEventSynchronize(p->ev[1]));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[0], p->ev[1]));
    p->prof_ms += ms;
    p->prof_launches += p->persistent ? 1 : (p->plane_order ? std::max(p->n[0], std::max(p->n[1], p->n[2])) : p->nstages);
    p->prof_updates += p->prof_pending_updates;
    ++p->prof_sweeps;
    p->prof_pending = false;
    return RT_OK;
}

// One formal solution over every active bin: the tile stages in order.  With
// timed set, each stage launch is bracketed by events (active_bins then counts the
// bins that do work, for the update tally).
// Sweep options beyond the plain formal solution: the moments mode (nq = 10) over a
// chunk of bins into its own partial-sum buffer with one wave per workgroup.
struct SweepMode {
    int nq = 1;
    int f0 = 0;
    int nfc = -1;
    void *part = nullptr;
    int waves = 0;
};

template <typename Real>
PlaneArgs<Real> plane_args(const rt_problem *p, const double *S)
{
    PlaneArgs<Real> A;
    for (int q = 0; q < 3; ++q) {
        A.n[q] = p->n[q];
        A.periodic[q] = p->periodic[q];
        A.bc_lo[q] = p->desc.bc_lo[q];
        A.bc_hi[q] = p->desc.bc_hi[q];
        A.tiles_a[q] = p->plane_tiles_a[q];
        A.ntiles[q] = p->plane_ntiles[q];
    }
    A.nf = p->nf;
    A.na = p->na;
    A.cells = p->cells;
    A.rays = p->d_rays;
    A.cls_off = p->d_cls_off;
    A.cls_rays = p->d_cls_rays;
    if constexpr (sizeof(Real) == 4)
        A.chi = p->chi32;
    else
        A.chi = p->chi64;
    A.S = S;
    A.B = p->B;
    for (int k = 0; k < 6; ++k) A.fixed[k] = p->desc.I_fixed[k];
    A.planes = static_cast<Real *>(p->planes);
    A.pmax = p->pmax;
    A.wrapI = p->wrapI;
    A.part = static_cast<Real *>(p->part);
    A.f0 = 0;
    A.nfc = p->nf;
    A.frozen = p->frozen;
    A.parity = p->parity;
    return A;
}

// One formal solution in plane order (quadratic upwind intensity): step t of every
// ray is one launch, t = 0 .. max(nx, ny, nz) - 1.
template <typename Real>
rt_status run_plane_sweep(rt_problem *p, const double *S, hipStream_t st, bool timed, int active_bins,
                          const SweepMode &mode)
{
    PlaneArgs<Real> A = plane_args<Real>(p, S);
    if (p->cold) {
        HIP_TRY(launch_plane_cold<Real>(A, st));
        p->cold = false;
    }
    if (mode.nfc > 0) {
        A.f0 = mode.f0;
        A.nfc = mode.nfc;
    }
    if (mode.part) A.part = static_cast<Real *>(mode.part);
    timed = timed && p->prof && !p->prof_pending && mode.nq == 1;
    const int steps = std::max(p->n[0], std::max(p->n[1], p->n[2]));
    for (int t = 0; t < steps; ++t) {
        if (timed && t == 0) HIP_TRY(hipEventRecord(p->ev[0], st));
        HIP_TRY(launch_plane_step<Real>(A, t, mode.nq, st));
        if (timed && t == steps - 1) HIP_TRY(hipEventRecord(p->ev[1], st));
    }
    if (timed) {
        p->prof_pending = true;
        p->prof_pending_updates = (double)p->cells * p->na * active_bins;
    }
    return RT_OK;
}

template <typename Real>
rt_status run_sweep(rt_problem *p, const double *S, hipStream_t st, bool timed = false, int active_bins = 0,
                    SweepMode mode = SweepMode())
{
    if (p->plane_order) return run_plane_sweep<Real>(p, S, st, timed, active_bins, mode);
    SweepArgs<Real> A = sweep_args<Real>(p, S);
    if (mode.nfc > 0) {
        A.f0 = mode.f0;
        A.nfc = mode.nfc;
    }
    if (mode.part) A.part = static_cast<Real *>(mode.part);
    if (p->cold) {
        HIP_TRY(launch_periodic_cold<Real>(A, st));
        p->cold = false;
    }
    HIP_TRY(launch_ghost_fill<Real>(A, st));
    timed = timed && p->prof && !p->prof_pending && mode.nq == 1;
    const int W = mode.waves > 0 ? mode.waves : p->waves;
    if (p->persistent && mode.nq == 1) {
        DagArgs D;
        D.counter = p->dag_counter;
        D.done = p->dag_done;
        D.err = p->flags + 2;
        D.wait_ticks = p->wait_ticks;
        D.ntiles = p->ntiles;
        D.nt0 = p->nt[0];
        D.nt1 = p->nt[1];
        A.stage_off = 0;
        A.stage_cnt = p->ntiles;
        // counters zeroed and the epoch advanced by a kernel (also under graph capture:
        // no memset node, and no epoch fixed at capture time)
        HIP_TRY(launch_dag_begin(p->dag_counter, st));
        if (timed) HIP_TRY(hipEventRecord(p->ev[0], st));
        if constexpr (sizeof(Real) == 8)
            HIP_TRY(launch_sweep_persistent_f64(A, D, W, p->bpo, st));
        else
            HIP_TRY(launch_sweep_persistent_f32(A, D, W, p->bpo, st));
        if (timed) {
            HIP_TRY(hipEventRecord(p->ev[1], st));
            p->prof_pending = true;
            p->prof_pending_updates = (double)p->cells * p->na * active_bins;
        }
        return RT_OK;
    }
    for (int s = 0; s < p->nstages; ++s) {
        A.stage_off = p->stage_off[s];
        A.stage_cnt = p->stage_off[s + 1] - p->stage_off[s];
        A.stage = s;
        if (timed && s == 0) HIP_TRY(hipEventRecord(p->ev[0], st));
        if constexpr (sizeof(Real) == 8)
            HIP_TRY(launch_sweep_stage_f64(A, W, mode.nq, st));
        else
            HIP_TRY(launch_sweep_stage_f32(A, W, mode.nq, st));
        if (timed && s == p->nstages - 1) HIP_TRY(hipEventRecord(p->ev[1], st));
    }
    if (timed) {
        p->prof_pending = true;
        p->prof_pending_updates = (double)p->cells * p->na * active_bins;
    }
    return RT_OK;
}

rt_status sweep_current_S(rt_problem *p, const double *S64, hipStream_t st, bool timed = false, int active = 0)
{
    if (p->f32) return run_sweep<float>(p, S64, st, timed, active);
    return run_sweep<double>(p, S64, st, timed, active);
}

// Start values of an ALI solve (section 5.1: J = B start, S = B; section 4: S from
// the previous J) and cleared per-bin control words.
rt_status ali_start(rt_problem *p, const rt_ali_opts *opts, double *S, const double *J, hipStream_t st)
{
    const int64_t nc = p->cells * p->nf;
    if (opts->warm_start == 0)
        HIP_TRY(hipMemcpyAsync(S, p->B, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    else if (opts->warm_start == 2)
        HIP_TRY(launch_warm_start(p->B, p->eps, J, S, nc, st));
    HIP_TRY(hipMemsetAsync(p->frozen, 0, sizeof(int) * p->nf, st));
    HIP_TRY(hipMemsetAsync(p->iters, 0, sizeof(int) * p->nf, st));
    HIP_TRY(hipMemsetAsync(p->flags, 0, sizeof(int) * 4, st));
    return RT_OK;
}

rt_status check_ali_opts(const rt_ali_opts *opts)
{
    if (opts->fixed_iters < 0) return fail(RT_E_INVALID, "fixed_iters must be >= 0");
    if (opts->fixed_iters == 0 && (opts->max_iter < 1 || !(opts->delta_c >= 0.0)))
        return fail(RT_E_INVALID, "need max_iter >= 1 and delta_c >= 0");
    if (opts->warm_start < 0 || opts->warm_start > 2) return fail(RT_E_INVALID, "warm_start must be 0, 1 or 2");
    return RT_OK;
}

AliCtl ctl_of(rt_problem *p)
{
    AliCtl c;
    c.frozen = p->frozen;
    c.parity = p->parity;
    c.iters = p->iters;
    c.resid = p->resid;
    c.blockmax = p->blockmax;
    c.nblk = kUpdateBlocks;
    c.flags = p->flags;
    return c;
}

// ---------------------------------------------------------------------------------
// Batched Jacobi ALI over independent problems on one stream.  Problems with the same
// sweep precision and waves per workgroup form a class; per iteration a class runs
// one ghost-value launch, one launch per stage index covering that stage of all its
// problems (grid y = problem), one update launch and one finalize launch, so the many
// small stages of small problems share launches.  Problems retire at the convergence
// checks and new ones can join there (the serving loop).
// ---------------------------------------------------------------------------------
struct BatchItem {
    rt_problem *p = nullptr;
    double *S = nullptr, *J = nullptr;
    rt_ali_opts opts{};
    int issued = 0;        // iterations issued so far
    int total = 0;         // fixed_iters, or max_iter
    bool nonfinite = false;
    rt_status err = RT_OK; // a sweep of this member failed (the persistent schedule's wait ran out)
    uint64_t tag = 0;      // caller's handle (batch index, server ticket)
};

int64_t ghost_entries(const rt_problem *p)
{
    int64_t t = 0;
    for (int q = 0; q < 3; ++q) {
        const int na_ = (q == 0) ? p->n[1] : p->n[0], nb_ = (q == 2) ? p->n[1] : p->n[2];
        t += (int64_t)(na_ + 1) * (nb_ + 1) + (int64_t)(p->nt[q] - 1) * (na_ + nb_ + 1);
    }
    return t;
}

class BatchRunner {
  public:
    explicit BatchRunner(hipStream_t st) : st_(st) {}
    ~BatchRunner()
    {
        for (Class &c : classes_) free_class(c);
        for (Class &c : spare_) free_class(c);
        if (d_done_) (void)hipFree(d_done_);
        if (h_done_) (void)hipHostFree(h_done_);
        if (d_err_) (void)hipFree(d_err_);
        if (h_err_) (void)hipHostFree(h_err_);
    }
    size_t size() const { return items_.size(); }
    const std::vector<BatchItem> &items() const { return items_; }

    // Queue start values and the cold periodic memory of a new member.
    rt_status add(const BatchItem &it)
    {
        rt_problem *p = it.p;
        rt_status s = ali_start(p, &it.opts, it.S, it.J, st_);
        if (s != RT_OK) return s;
        if (p->cold && !p->plane_order) {   // a plane-ordered member's first sweep fills its own
            if (p->f32)
                HIP_TRY(launch_periodic_cold<float>(sweep_args<float>(p, it.S), st_));
            else
                HIP_TRY(launch_periodic_cold<double>(sweep_args<double>(p, it.S), st_));
            p->cold = false;
        }
        items_.push_back(it);
        dirty_ = true;
        return RT_OK;
    }

    // Issue the next iterations of every member (up to `every`, never past a member's
    // total), then read the stop flags (synchronises the stream).  Members that stopped
    // or reached their total move to `finished`.
    rt_status chunk(int every, std::vector<BatchItem> &finished)
    {
        if (items_.empty()) return RT_OK;
        if (dirty_) {
            rt_status s = rebuild();
            if (s != RT_OK) return s;
        }
        int k = every;
        for (const BatchItem &it : items_) k = std::min(k, it.total - it.issued);
        k = std::max(k, 1);
        for (int j = 0; j < k; ++j)
            for (Class &c : classes_) {
                const int n = (int)c.idx.size();
                if (c.plane) {
                    // a plane-ordered member on its own: its sweep (one launch per plane
                    // step), the update over its 24 class slots, the batch's convergence launch
                    const BatchItem &it = items_[c.idx[0]];
                    rt_problem *p = it.p;
                    const AliCtl ctl = c.h_upd[0].ctl;
                    rt_status s = sweep_current_S(p, it.S, st_);
                    if (s != RT_OK) return s;
                    if (p->f32)
                        HIP_TRY(launch_ali_update<float>(static_cast<float *>(p->part), p->npart, 1, p->nf, p->cells,
                                                         p->B, p->eps, p->lam, it.S, it.J, ctl, st_));
                    else
                        HIP_TRY(launch_ali_update<double>(static_cast<double *>(p->part), p->npart, 0, p->nf, p->cells,
                                                          p->B, p->eps, p->lam, it.S, it.J, ctl, st_));
                    HIP_TRY(launch_ali_finalize_batch(c.d_upd, 1, d_done_ + 2 * c.done_off, st_));
                    continue;
                }
                if (c.f32) {
                    const SweepArgs<float> *a = static_cast<const SweepArgs<float> *>(c.d_args);
                    HIP_TRY(launch_ghost_fill_batch<float>(a, n, c.max_ghost, c.max_na, st_));
                    if (c.persist)
                        HIP_TRY(launch_sweep_persistent_batch_f32(a, c.d_mem, c.d_items, c.nitems, n, c.d_dag, d_err_,
                                                                  c.wait_ticks, c.waves, c.bpo, st_));
                    else
                        for (size_t st = 0; st < c.max_items.size(); ++st)
                            HIP_TRY(launch_sweep_batch_stage_f32(a, n, (int)st, c.max_items[st], c.waves, c.multi,
                                                                 c.order, st_));
                    HIP_TRY(launch_ali_update_batch<float>(c.d_upd, n, kBatchUpdateBlocks, c.max_nf, st_));
                } else {
                    const SweepArgs<double> *a = static_cast<const SweepArgs<double> *>(c.d_args);
                    HIP_TRY(launch_ghost_fill_batch<double>(a, n, c.max_ghost, c.max_na, st_));
                    if (c.persist)
                        HIP_TRY(launch_sweep_persistent_batch_f64(a, c.d_mem, c.d_items, c.nitems, n, c.d_dag, d_err_,
                                                                  c.wait_ticks, c.waves, c.bpo, st_));
                    else
                        for (size_t st = 0; st < c.max_items.size(); ++st)
                            HIP_TRY(launch_sweep_batch_stage_f64(a, n, (int)st, c.max_items[st], c.waves, c.multi,
                                                                 c.order, st_));
                    HIP_TRY(launch_ali_update_batch<double>(c.d_upd, n, kBatchUpdateBlocks, c.max_nf, st_));
                }
                HIP_TRY(launch_ali_finalize_batch(c.d_upd, n, d_done_ + 2 * c.done_off, st_));
            }
        for (BatchItem &it : items_) it.issued += k;
        HIP_TRY(hipMemcpyAsync(h_done_, d_done_, sizeof(int) * 2 * items_.size(), hipMemcpyDeviceToHost, st_));
        HIP_TRY(hipMemcpyAsync(h_err_, d_err_, sizeof(int), hipMemcpyDeviceToHost, st_));
        HIP_TRY(hipStreamSynchronize(st_));
        // a dependency wait of a persistent sweep ran out: the members of the persistent
        // classes leave the batch with RT_E_HIP (the flag does not say which class), the
        // others go on
        const bool wait_failed = *h_err_ != 0;
        if (wait_failed) {
            HIP_TRY(hipMemsetAsync(d_err_, 0, sizeof(int), st_));
            HIP_TRY(hipStreamSynchronize(st_));
            *h_err_ = 0;
        }
        std::vector<int> pos(items_.size());   // member -> its slot in the flag array
        std::vector<char> persist(items_.size(), 0);
        for (const Class &c : classes_)
            for (size_t j = 0; j < c.idx.size(); ++j) {
                pos[c.idx[j]] = c.done_off + (int)j;
                persist[c.idx[j]] = c.persist;
            }
        std::vector<BatchItem> keep;
        for (size_t i = 0; i < items_.size(); ++i) {
            BatchItem it = items_[i];
            const int g = pos[i];
            it.nonfinite = h_done_[2 * g + 1] != 0;
            if (wait_failed && persist[i]) it.err = RT_E_HIP;
            if (it.err != RT_OK || h_done_[2 * g] || it.issued >= it.total)
                finished.push_back(it);
            else
                keep.push_back(it);
        }
        if (keep.size() != items_.size()) dirty_ = true;
        items_.swap(keep);
        if (dirty_ && !items_.empty()) return rebuild();   // class indices follow the new order
        return RT_OK;
    }

  private:
    struct Class {
        bool f32 = false;
        bool plane = false;                   // one plane-ordered member, launches of its own
        int waves = 1;
        bool multi = false;
        int order = 0;
        std::vector<int> idx;                 // members (positions in items_)
        std::vector<unsigned char> h_args;    // SweepArgs<Real> per member
        std::vector<BatchUpdate> h_upd;
        void *d_args = nullptr;
        BatchUpdate *d_upd = nullptr;
        size_t cap = 0;                       // members the device arrays hold
        std::vector<int> max_items;           // per stage index: max workgroups over members
        int64_t max_ghost = 0;
        int max_na = 0, max_nf = 0, done_off = 0;
        // persistent schedule: the whole sweep of every member in one launch
        bool persist = false;
        std::vector<PersistItem> h_items;
        std::vector<PersistMember> h_mem;
        PersistItem *d_items = nullptr;
        PersistMember *d_mem = nullptr;
        int *d_dag = nullptr;                 // [8] ticket counters of the octants
        size_t items_cap = 0, mem_cap = 0;
        int nitems = 0, bpo = 1;
        uint64_t wait_ticks = 0;
    };
    hipStream_t st_;
    std::vector<BatchItem> items_;
    std::vector<Class> classes_, spare_;
    int *d_done_ = nullptr;
    int *h_done_ = nullptr;
    size_t done_cap_ = 0;
    int *d_err_ = nullptr;      // set by a persistent sweep whose dependency wait ran out
    int *h_err_ = nullptr;
    bool dirty_ = true;

    static void free_class(Class &c)
    {
        if (c.d_args) (void)hipFree(c.d_args);
        if (c.d_upd) (void)hipFree(c.d_upd);
        c.d_args = nullptr;
        c.d_upd = nullptr;
        c.cap = 0;
        free_persist(c);
    }

    static void free_persist(Class &c)
    {
        if (c.d_items) (void)hipFree(c.d_items);
        if (c.d_mem) (void)hipFree(c.d_mem);
        if (c.d_dag) (void)hipFree(c.d_dag);
        c.d_items = nullptr;
        c.d_mem = nullptr;
        c.d_dag = nullptr;
        c.items_cap = c.mem_cap = 0;
    }

    // Work list of a persistent class: stage by stage, then member, bin and tile, so
    // upwind neighbours always come first (and are drawn earlier).
    rt_status build_persist(Class &c)
    {
        const size_t n = c.idx.size();
        c.h_mem.resize(n);
        c.h_items.clear();
        int max_stages = 0;
        for (size_t j = 0; j < n; ++j) {
            rt_problem *p = items_[c.idx[j]].p;
            PersistMember &m = c.h_mem[j];
            m.done = p->dag_done;
            m.counter = p->dag_counter;
            m.ntiles = p->ntiles;
            m.nt0 = p->nt[0];
            m.nt1 = p->nt[1];
            m.pad = 0;
            max_stages = std::max(max_stages, p->nstages);
        }
        for (int s2 = 0; s2 < max_stages; ++s2)
            for (size_t j = 0; j < n; ++j) {
                const rt_problem *p = items_[c.idx[j]].p;
                if (s2 >= p->nstages) continue;
                for (int f = 0; f < p->nf; ++f)
                    for (int z = p->stage_off[s2]; z < p->stage_off[s2 + 1]; ++z)
                        c.h_items.push_back(PersistItem{(int)j, f, z, 0});
            }
        if (c.h_items.size() > (size_t)INT32_MAX) return fail(RT_E_UNSUPPORTED, "persistent batch: too many tiles");
        c.nitems = (int)c.h_items.size();
        hipError_t e = hipSuccess;
        if (!c.d_dag) {
            e = hipMalloc((void **)&c.d_dag, sizeof(int) * 16);
            if (e == hipSuccess) e = hipMemsetAsync(c.d_dag, 0, sizeof(int) * 16, st_);
        }
        if (e == hipSuccess && c.items_cap < c.h_items.size()) {
            if (c.d_items) (void)hipFree(c.d_items);
            c.d_items = nullptr;
            c.items_cap = 0;
            e = hipMalloc((void **)&c.d_items, sizeof(PersistItem) * std::max<size_t>(c.h_items.size(), 1));
            if (e == hipSuccess) c.items_cap = c.h_items.size();
        }
        if (e == hipSuccess && c.mem_cap < n) {
            if (c.d_mem) (void)hipFree(c.d_mem);
            c.d_mem = nullptr;
            c.mem_cap = 0;
            e = hipMalloc((void **)&c.d_mem, sizeof(PersistMember) * std::max<size_t>(n, 8));
            if (e == hipSuccess) c.mem_cap = std::max<size_t>(n, 8);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_persist(c);
            return fail(RT_E_OOM, "persistent batch work list allocation failed");
        }
        if (c.nitems > 0)
            HIP_TRY(hipMemcpyAsync(c.d_items, c.h_items.data(), sizeof(PersistItem) * c.h_items.size(),
                                   hipMemcpyHostToDevice, st_));
        HIP_TRY(hipMemcpyAsync(c.d_mem, c.h_mem.data(), sizeof(PersistMember) * n, hipMemcpyHostToDevice, st_));
        int dev = 0, per_cu = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            persistent_batch_blocks_per_cu(c.f32 ? 4 : 8, c.waves, &per_cu) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 8) ncu = 8;
        (void)hipGetLastError();
        c.bpo = std::max(1, std::min(per_cu * ncu / 8, c.nitems));
        c.wait_ticks = 0;
        for (size_t j = 0; j < n; ++j) c.wait_ticks = std::max(c.wait_ticks, items_[c.idx[j]].p->wait_ticks);
        return RT_OK;
    }

    template <typename Real>
    void fill_args(Class &c)
    {
        c.h_args.assign(c.idx.size() * sizeof(SweepArgs<Real>), 0);
        SweepArgs<Real> *a = reinterpret_cast<SweepArgs<Real> *>(c.h_args.data());
        for (size_t j = 0; j < c.idx.size(); ++j) {
            const BatchItem &it = items_[c.idx[j]];
            a[j] = sweep_args<Real>(it.p, it.S);
        }
    }

    rt_status rebuild()
    {
        // keep the device arrays of the old classes for reuse
        for (Class &c : classes_) {
            c.idx.clear();
            spare_.push_back(std::move(c));
        }
        classes_.clear();
        for (size_t i = 0; i < items_.size(); ++i) {
            const rt_problem *p = items_[i].p;
            const bool multi = p->R > p->waves;
            Class *cls = nullptr;
            if (!p->plane_order)
                for (Class &c : classes_)
                    if (!c.plane && c.f32 == p->f32 && c.waves == p->waves && c.multi == multi &&
                        c.order == p->desc.order && c.persist == p->persistent)
                        cls = &c;
            if (!cls) {
                Class c;
                if (!spare_.empty()) {
                    c = std::move(spare_.back());
                    spare_.pop_back();
                }
                c.plane = p->plane_order;
                c.f32 = p->f32;
                c.waves = p->waves;
                c.multi = multi;
                c.order = p->desc.order;
                c.persist = p->persistent;
                classes_.push_back(std::move(c));
                cls = &classes_.back();
            }
            cls->idx.push_back((int)i);
        }
        int off = 0;
        for (Class &c : classes_) {
            const size_t n = c.idx.size();
            if (c.f32)
                fill_args<float>(c);
            else
                fill_args<double>(c);
            c.h_upd.resize(n);
            c.max_items.clear();
            c.max_ghost = 0;
            c.max_na = c.max_nf = 0;
            for (size_t j = 0; j < n; ++j) {
                const BatchItem &it = items_[c.idx[j]];
                rt_problem *p = it.p;
                BatchUpdate &u = c.h_upd[j];
                u.part = p->part;
                u.B = p->B;
                u.eps = p->eps;
                u.lam = p->lam;
                u.S64 = it.S;
                u.J = it.J;
                u.cells = p->cells;
                u.nf = p->nf;
                u.dform = p->f32 ? 1 : 0;
                u.ctl = ctl_of(p);
                u.ctl.nblk = kBatchUpdateBlocks;
                u.fixed_mode = it.opts.fixed_iters > 0 ? 1 : 0;
                u.delta_c = it.opts.delta_c;
                u.per_bin_stop = it.opts.per_bin_stop ? 1 : 0;
                if ((int)c.max_items.size() < p->nstages) c.max_items.resize(p->nstages, 0);
                for (int s2 = 0; s2 < p->nstages; ++s2)
                    c.max_items[s2] = std::max(c.max_items[s2], (p->stage_off[s2 + 1] - p->stage_off[s2]) * 8 * p->nf);
                c.max_ghost = std::max(c.max_ghost, ghost_entries(p));
                c.max_na = std::max(c.max_na, p->na);
                c.max_nf = std::max(c.max_nf, p->nf);
            }
            if (c.cap < n) {
                free_class(c);
                const size_t cap = std::max<size_t>(n, 8);
                const size_t asz = c.f32 ? sizeof(SweepArgs<float>) : sizeof(SweepArgs<double>);
                hipError_t e = hipMalloc(&c.d_args, cap * std::max(sizeof(SweepArgs<float>), sizeof(SweepArgs<double>)));
                if (e == hipSuccess) e = hipMalloc((void **)&c.d_upd, cap * sizeof(BatchUpdate));
                (void)asz;
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    free_class(c);
                    return fail(RT_E_OOM, "batch descriptor allocation failed");
                }
                c.cap = cap;
            }
            HIP_TRY(hipMemcpyAsync(c.d_args, c.h_args.data(), c.h_args.size(), hipMemcpyHostToDevice, st_));
            HIP_TRY(hipMemcpyAsync(c.d_upd, c.h_upd.data(), n * sizeof(BatchUpdate), hipMemcpyHostToDevice, st_));
            if (c.persist) {
                rt_status ps = build_persist(c);
                if (ps != RT_OK) return ps;
            }
            c.done_off = off;
            off += (int)n;
        }
        if (done_cap_ < items_.size()) {
            if (d_done_) (void)hipFree(d_done_);
            if (h_done_) (void)hipHostFree(h_done_);
            d_done_ = nullptr;
            h_done_ = nullptr;
            const size_t cap = std::max<size_t>(items_.size(), 64);
            hipError_t e = hipMalloc((void **)&d_done_, sizeof(int) * 2 * cap);
            if (e == hipSuccess) e = hipHostMalloc((void **)&h_done_, sizeof(int) * 2 * cap, hipHostMallocDefault);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                done_cap_ = 0;
                return fail(RT_E_OOM, "batch flag allocation failed");
            }
            done_cap_ = cap;
        }
        if (!d_err_) {
            hipError_t e = hipMalloc((void **)&d_err_, sizeof(int));
            if (e == hipSuccess) e = hipHostMalloc((void **)&h_err_, sizeof(int), hipHostMallocDefault);
            if (e == hipSuccess) e = hipMemsetAsync(d_err_, 0, sizeof(int), st_);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                if (d_err_) (void)hipFree(d_err_);
                d_err_ = nullptr;
                return fail(RT_E_OOM, "batch flag allocation failed");
            }
            *h_err_ = 0;
        }
        // host arrays must outlive the copies: wait for them here
        HIP_TRY(hipStreamSynchronize(st_));
        dirty_ = false;
        return RT_OK;
    }
};

// Per-problem results of an ALI solve, read from the device (synchronises).
rt_status ali_stats(rt_problem *p, const rt_ali_opts *opts, bool nonfinite, double seconds, rt_ali_stats *stats,
                    hipStream_t st, rt_status *result)
{
    std::vector<int> iters(p->nf);
    std::vector<double> resid(p->nf);
    HIP_TRY(hipMemcpyAsync(iters.data(), p->iters, sizeof(int) * p->nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(resid.data(), p->resid, sizeof(double) * p->nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int conv = 0, maxit = 0;
    double maxr = 0.0;
    for (int f = 0; f < p->nf; ++f) {
        conv += resid[f] <= opts->delta_c;
        maxit = std::max(maxit, iters[f]);
        maxr = std::max(maxr, resid[f]);
    }
    if (stats) {
        stats->iterations = maxit;
        stats->bins_converged = conv;
        stats->max_rel_dS = maxr;
        stats->seconds = seconds;
    }
    if (nonfinite)
        *result = RT_E_NONFINITE;
    else if (opts->fixed_iters == 0 && conv < p->nf)
        *result = RT_NOT_CONVERGED;
    else
        *result = RT_OK;
    return RT_OK;
}

}  // namespace

namespace rtsc {

// for the no-allocation formal solution (rt_noalloc.hip)
rt_status validate_desc(const rt_problem_desc *d, int *na_out) { return validate(d, na_out); }
void record_error(const char *msg) { (void)fail(RT_OK, "%s", msg); }

}  // namespace rtsc

extern "C" {

const char *rt_status_string(rt_status s)
{
    switch (s) {
    case RT_OK: return "ok";
    case RT_NOT_CONVERGED: return "not converged";
    case RT_E_INVALID: return "invalid argument";
    case RT_E_OOM: return "out of device memory";
    case RT_E_HIP: return "HIP runtime error";
    case RT_E_NONFINITE: return "non-finite residual";
    case RT_E_UNSUPPORTED: return "unsupported";
    case RT_E_BUSY: return "busy";
    }
    return "unknown status";
}

const char *rt_last_error(const rt_context *ctx)
{
    if (!ctx) return g_err.c_str();
    thread_local std::string copy;
    {
        std::lock_guard<std::mutex> lk(const_cast<rt_context *>(ctx)->mu);
        copy = ctx->err;
    }
    return copy.c_str();
}

rt_status rt_context_create(int32_t device, rt_context **out)
{
    if (!out) return fail(RT_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) {
        (void)hipGetLastError();
        count = 0;
    }
    if (device < 0 || device >= count) return fail(RT_E_INVALID, "no HIP device %d (%d visible)", device, count);
    rt_context *c = new rt_context();
    c->device = device;
    *out = c;
    return RT_OK;
}

rt_status rt_context_destroy(rt_context *ctx)
{
    delete ctx;
    return RT_OK;
}

rt_status rt_quadrature(int32_t n_mu, double *mu_out, double *w_out, int32_t *na_out)
{
    if (n_mu != 2 && n_mu != 4 && n_mu != 6 && n_mu != 8 && n_mu != 10 && n_mu != 12)
        return fail(RT_E_INVALID, "n_mu must be 2, 4, 6, 8, 10 or 12");
    const int na = n_mu * (n_mu + 2);
    if (na_out) *na_out = na;
    if (!mu_out && !w_out) return RT_OK;
    std::vector<double> mu, w;
    if (!level_symmetric(n_mu, mu, w)) return fail(RT_E_INVALID, "no level-symmetric set for n_mu=%d", n_mu);
    if ((int)w.size() != na) return fail(RT_E_INVALID, "internal: %zu rays for n_mu=%d", w.size(), n_mu);
    if (mu_out) std::memcpy(mu_out, mu.data(), sizeof(double) * mu.size());
    if (w_out) std::memcpy(w_out, w.data(), sizeof(double) * w.size());
    return RT_OK;
}

rt_status rt_problem_bytes(const rt_problem_desc *desc, size_t *bytes)
{
    int na;
    rt_status s = validate(desc, &na);
    if (s != RT_OK) return s;
    if (!bytes) return fail(RT_E_INVALID, "bytes is NULL");
    *bytes = state_bytes(desc, na);
    return RT_OK;
}

rt_status rt_problem_destroy(rt_problem *p)
{
    if (!p) return RT_OK;
    CallScope scope(p->ctx, p->device);
    // a server's worker may still launch kernels on its state
    if (p->server_refs.load() > 0) return fail(RT_E_BUSY, "the problem has a queued or running server request");
    for (void *v : p->allocs) (void)hipFree(v);
    if (p->h_flags) (void)hipHostFree(p->h_flags);
    if (p->h_sum) (void)hipHostFree(p->h_sum);
    if (p->h_frozen) (void)hipHostFree(p->h_frozen);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : p->gs_ev) (void)hipEventDestroy(e);
    for (auto &g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    delete p;
    return RT_OK;
}

rt_status rt_problem_create(rt_context *ctx, const rt_problem_desc *desc, rt_problem **out)
{
    CallScope scope(ctx, ctx ? ctx->device : -1);
    if (!out) return fail(RT_E_INVALID, "out is NULL");
    *out = nullptr;
    int na;
    rt_status s = validate(desc, &na);
    if (s != RT_OK) return s;

    rt_problem *p = new rt_problem();
    p->ctx = ctx;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(RT_E_HIP, "no current HIP device");
    }
    p->usr32 = desc->in_dtype == RT_DTYPE_F32;
    p->desc = *desc;
    p->desc.mu = nullptr;
    p->desc.w = nullptr;
    p->desc.w_nu = nullptr;
    p->n[0] = desc->nx;
    p->n[1] = desc->ny;
    p->n[2] = desc->nz;
    p->nf = desc->nf;
    p->na = na;
    p->R = na / 8;
    p->f32 = desc->precision == RT_F32;
    p->cells = (int64_t)desc->nx * desc->ny * desc->nz;
    p->plane[0] = (int64_t)desc->ny * desc->nz;
    p->plane[1] = (int64_t)desc->nx * desc->nz;
    p->plane[2] = (int64_t)desc->nx * desc->ny;
    p->pplane[0] = FacePlane(desc->ny, desc->nz).slot();
    p->pplane[1] = FacePlane(desc->nx, desc->nz).slot();
    p->pplane[2] = FacePlane(desc->nx, desc->ny).slot();
    for (int q = 0; q < 3; ++q) p->periodic[q] = desc->bc_lo[q] == RT_BC_PERIODIC;
    tile_counts(desc, p->nt);
    p->w_nu.assign(desc->nf, 1.0);
    if (desc->w_nu) std::copy(desc->w_nu, desc->w_nu + desc->nf, p->w_nu.begin());

    // rays, grouped by octant (stable within an octant)
    std::vector<double> mu, w;
    if (desc->mu) {
        mu.assign(desc->mu, desc->mu + 3 * na);
        w.assign(desc->w, desc->w + na);
    } else if (!level_symmetric(desc->n_mu, mu, w)) {
        delete p;
        return fail(RT_E_INVALID, "no level-symmetric set for n_mu=%d", desc->n_mu);
    }
    const double h[3] = {desc->dx, desc->dy, desc->dz};
    for (int o = 0; o < 8; ++o)
        for (int k = 0; k < na; ++k)
            if (octant_of(&mu[3 * k]) == o) p->rays.push_back(ray_geometry(&mu[3 * k], h, w[k], k));

    // tile schedule: tiles sorted by stage tx + ty + tz
    p->nstages = p->nt[0] + p->nt[1] + p->nt[2] - 2;
    std::vector<int> tiles;
    p->stage_off.assign(p->nstages + 1, 0);
    for (int s2 = 0; s2 < p->nstages; ++s2) {
        p->stage_off[s2] = (int)tiles.size();
        for (int tz = 0; tz < p->nt[2]; ++tz)
            for (int ty = 0; ty < p->nt[1]; ++ty) {
                const int tx = s2 - ty - tz;
                if (tx >= 0 && tx < p->nt[0]) tiles.push_back(tx | (ty << 10) | (tz << 20));
            }
    }
    p->stage_off[p->nstages] = (int)tiles.size();
    // RTSC_TILE_ORDER_SEED = n != 0: the tiles of every stage in a pseudo-random order
    // seeded with n.  Tiles of one stage are independent, so results stay bitwise the
    // same; a test of that checks the schedule for races.
    if (const char *seed = std::getenv("RTSC_TILE_ORDER_SEED")) {
        const unsigned long long v = std::strtoull(seed, nullptr, 10);
        if (v != 0) {
            std::mt19937_64 gen(v);
            for (int s2 = 0; s2 < p->nstages; ++s2)
                std::shuffle(tiles.begin() + p->stage_off[s2], tiles.begin() + p->stage_off[s2 + 1], gen);
        }
    }

    const int64_t nc = p->cells * p->nf;
    const size_t rs = real_size(desc);
#define ALLOC(ptr, cnt)                         \
    do {                                        \
        rt_status a_ = dalloc(p, &(ptr), (cnt)); \
        if (a_ != RT_OK) {                      \
            rt_problem_destroy(p);              \
            return a_;                          \
        }                                       \
    } while (0)
    ALLOC(p->d_rays, (size_t)na);
    ALLOC(p->d_tiles, tiles.size());
    ALLOC(p->d_stage_tab, p->stage_off.size());
    ALLOC(p->chi64, (size_t)nc);
    ALLOC(p->eps, (size_t)nc);
    ALLOC(p->B, (size_t)nc);
    ALLOC(p->lam, (size_t)nc);
    if (p->f32) ALLOC(p->chi32, (size_t)nc);
    if (p->usr32) {
        ALLOC(p->stS, (size_t)nc);
        ALLOC(p->stJ, (size_t)nc);
    }
    p->plane_order = desc->interp == RT_INTERP_QUADRATIC;
    p->npart = p->plane_order ? kPlaneParts : 8;
    if (p->plane_order) {
        p->pmax = std::max(p->plane[0], std::max(p->plane[1], p->plane[2]));
        unsigned char *pl;
        ALLOC(pl, (size_t)p->nf * na * 2 * p->pmax * rs);
        p->planes = pl;
        if (p->f32) ALLOC(p->wrapI, (size_t)p->nf * na * p->pmax);
        ALLOC(p->d_cls_off, (size_t)kPlaneParts + 1);
        ALLOC(p->d_cls_rays, (size_t)na);
        for (int q = 0; q < 3; ++q) {
            const int a = q == 0 ? 1 : 0, b = q == 2 ? 1 : 2;
            p->plane_tiles_a[q] = (p->n[a] + kPlaneTile - 1) / kPlaneTile;
            p->plane_ntiles[q] = p->plane_tiles_a[q] * ((p->n[b] + kPlaneTile - 1) / kPlaneTile);
        }
    } else {
        for (int q = 0; q < 3; ++q) {
            unsigned char *fb;
            ALLOC(fb, (size_t)p->nf * na * p->nt[q] * p->pplane[q] * rs);
            p->face[q] = fb;
            if (p->periodic[q]) ALLOC(p->wrap[q], (size_t)p->nf * na * 2 * p->plane[q]);
        }
    }
    {
        unsigned char *pb;
        ALLOC(pb, (size_t)p->npart * nc * rs);
        p->part = pb;
    }
    ALLOC(p->frozen, (size_t)p->nf);
    ALLOC(p->parity, (size_t)p->nf);
    ALLOC(p->iters, (size_t)p->nf);
    ALLOC(p->resid, (size_t)p->nf);
    ALLOC(p->blockmax, (size_t)p->nf * kUpdateBlocks);
    ALLOC(p->flags, 4);
    p->ntiles = p->nt[0] * p->nt[1] * p->nt[2];
    ALLOC(p->dag_counter, 16);
    ALLOC(p->dag_done, (size_t)p->nf * 8 * p->ntiles);
#undef ALLOC
    if (hipHostMalloc((void **)&p->h_flags, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&p->h_frozen, sizeof(int) * p->nf, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p->h_flags = nullptr;
        rt_problem_destroy(p);
        return fail(RT_E_OOM, "pinned host allocation failed");
    }
    int dev = 0, lds_limit = 65536;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    (void)hipGetLastError();
    p->waves = sweep_waves(p->R, p->f32, desc->order, (size_t)lds_limit);
    p->lds_limit = (size_t)lds_limit;
    p->persistent = desc->schedule == RT_SCHED_PERSISTENT;
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        (void)hipGetLastError();
        p->wall_khz = khz;
        p->wait_ticks = (uint64_t)khz * 20;   // 20 ms
    }
    if (p->persistent) persistent_grid(p);
    if (sweep_lds_bytes(p->f32 ? 4 : 8, p->waves, 1, p->R > p->waves, desc->order) > (size_t)lds_limit) {
        rt_problem_destroy(p);
        return fail(RT_E_UNSUPPORTED, "sweep needs %zu bytes of LDS, device allows %d",
                    sweep_lds_bytes(p->f32 ? 4 : 8, p->waves, 1, p->R > p->waves, desc->order), lds_limit);
    }
    hipError_t e = hipMemcpy(p->d_rays, p->rays.data(), sizeof(RayGeo) * na, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_tiles, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_stage_tab, p->stage_off.data(), sizeof(int) * p->stage_off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(p->frozen, 0, sizeof(int) * p->nf);
    if (e == hipSuccess) e = hipMemset(p->parity, 0, sizeof(int) * p->nf);
    if (e == hipSuccess) e = hipMemset(p->flags, 0, sizeof(int) * 4);
    if (e == hipSuccess) e = hipMemset(p->dag_done, 0, sizeof(int) * (size_t)p->nf * 8 * p->ntiles);
    if (e == hipSuccess) e = hipMemset(p->dag_counter, 0, sizeof(int) * 16);   // tickets and the epoch
    if (e == hipSuccess && p->plane_order) {
        // classes (octant, first-crossed axis); a class without rays keeps zero partials
        std::vector<int> off(kPlaneParts + 1, 0), list;
        for (int c = 0; c < kPlaneParts; ++c) {
            off[c] = (int)list.size();
            for (int k = 0; k < na; ++k)
                if (p->rays[k].oct * 3 + p->rays[k].d == c) list.push_back(k);
        }
        off[kPlaneParts] = (int)list.size();
        e = hipMemcpy(p->d_cls_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->d_cls_rays, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(p->part, 0, (size_t)p->npart * nc * rs);
    }
    if (e != hipSuccess) {
        rt_problem_destroy(p);
        return fail(RT_E_HIP, "problem initialisation failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return RT_OK;
}

rt_status rt_problem_set_fields(rt_problem *p, const void *chi, const void *eps, const void *B, void *stream)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    if (!chi || !eps || !B) return fail(RT_E_INVALID, "chi, eps and B are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nc = p->cells * p->nf;
    if (p->usr32) {
        HIP_TRY(launch_convert_f64(static_cast<const float *>(chi), p->chi64, nc, st));
        HIP_TRY(launch_convert_f64(static_cast<const float *>(eps), p->eps, nc, st));
        HIP_TRY(launch_convert_f64(static_cast<const float *>(B), p->B, nc, st));
    } else {
        const size_t bytes = sizeof(double) * nc;
        HIP_TRY(hipMemcpyAsync(p->chi64, chi, bytes, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(p->eps, eps, bytes, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(p->B, B, bytes, hipMemcpyDeviceToDevice, st));
    }
    if (p->f32) HIP_TRY(launch_convert_f32(p->chi64, p->chi32, p->cells * p->nf, st));
    HIP_TRY(launch_lambda_star(p->n, p->desc.bc_lo, p->desc.bc_hi, p->nf, p->na, p->desc.order, p->d_rays, p->chi64,
                               p->lam, st));
    HIP_TRY(hipMemsetAsync(p->parity, 0, sizeof(int) * p->nf, st));
    p->cold = true;
    p->have_fields = true;
    return RT_OK;
}

rt_status rt_problem_reset_periodic(rt_problem *p, void *stream)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    HIP_TRY(hipMemsetAsync(p->parity, 0, sizeof(int) * p->nf, static_cast<hipStream_t>(stream)));
    p->cold = true;
    return RT_OK;
}

}  // extern "C"

namespace {

// Saved periodic memory: this header, the per-bin slot selectors, then the buffers
// the next sweep may read, each padded to 256 bytes.
struct StateHeader {
    char magic[8];
    int32_t n[3], nf, na, f32, plane_order, periodic, cold;
    uint32_t rays;    // FNV-1a hash of the rays' direction cosines and weights, in sweep order
    int64_t bytes;
};
static_assert(sizeof(StateHeader) == 56, "saved-state header layout");
constexpr char kStateMagic[8] = {'R', 'T', 'S', 'C', 'S', 'T', '0', '1'};

inline size_t pad256(size_t b) { return (b + 255) & ~size_t(255); }

// The device buffers that carry the periodic memory from one sweep to the next.
std::vector<std::pair<void *, size_t>> state_buffers(rt_problem *p)
{
    std::vector<std::pair<void *, size_t>> v;
    v.push_back({p->parity, sizeof(int) * p->nf});
    const size_t rs = p->f32 ? 4 : 8;
    if (p->plane_order) {
        v.push_back({p->planes, (size_t)p->nf * p->na * 2 * p->pmax * rs});
        if (p->wrapI) v.push_back({p->wrapI, (size_t)p->nf * p->na * p->pmax * 8});
    } else {
        for (int q = 0; q < 3; ++q)
            if (p->wrap[q]) v.push_back({p->wrap[q], (size_t)p->nf * p->na * 2 * p->plane[q] * 8});
    }
    return v;
}

StateHeader state_header(rt_problem *p)
{
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    for (int q = 0; q < 3; ++q) h.n[q] = p->n[q];
    h.nf = p->nf;
    h.na = p->na;
    h.f32 = p->f32;
    h.plane_order = p->plane_order;
    h.periodic = p->periodic[0] | p->periodic[1] << 1 | p->periodic[2] << 2;
    h.cold = p->cold;
    uint32_t fnv = 2166136261u;
    for (const RayGeo &g : p->rays) {
        const double v[4] = {g.mu[0], g.mu[1], g.mu[2], g.wk};
        const unsigned char *c = reinterpret_cast<const unsigned char *>(v);
        for (size_t i = 0; i < sizeof v; ++i) fnv = (fnv ^ c[i]) * 16777619u;
    }
    h.rays = fnv;
    h.bytes = (int64_t)pad256(sizeof(StateHeader));
    for (auto &b : state_buffers(p)) h.bytes += (int64_t)pad256(b.second);
    return h;
}

}  // namespace

extern "C" {

rt_status rt_problem_state_bytes(rt_problem *p, size_t *bytes)
{
    if (!p || !bytes) return fail(RT_E_INVALID, "problem and bytes are required");
    CallScope scope(p->ctx, p->device);
    *bytes = (size_t)state_header(p).bytes;
    return RT_OK;
}

rt_status rt_problem_save_state(rt_problem *p, void *dst, size_t bytes, void *stream)
{
    if (!p || !dst) return fail(RT_E_INVALID, "problem and dst are required");
    CallScope scope(p->ctx, p->device);
    const StateHeader h = state_header(p);
    if (bytes < (size_t)h.bytes) return fail(RT_E_INVALID, "dst holds %zu bytes, the state needs %lld", bytes,
                                             (long long)h.bytes);
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    unsigned char *o = static_cast<unsigned char *>(dst);
    HIP_TRY(hipMemcpy(o, &h, sizeof h, hipMemcpyDefault));
    size_t off = pad256(sizeof h);
    for (auto &b : state_buffers(p)) {
        HIP_TRY(hipMemcpy(o + off, b.first, b.second, hipMemcpyDefault));
        off += pad256(b.second);
    }
    return RT_OK;
}

rt_status rt_problem_load_state(rt_problem *p, const void *src, size_t bytes, void *stream)
{
    if (!p || !src) return fail(RT_E_INVALID, "problem and src are required");
    CallScope scope(p->ctx, p->device);
    if (bytes < sizeof(StateHeader)) return fail(RT_E_INVALID, "src holds %zu bytes, less than a header", bytes);
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    StateHeader h;
    HIP_TRY(hipMemcpy(&h, src, sizeof h, hipMemcpyDefault));
    const StateHeader mine = state_header(p);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(RT_E_INVALID, "src is not a saved problem state");
    const bool cold = h.cold != 0;
    h.cold = mine.cold;   // the one field that may differ
    if (std::memcmp(&h, &mine, sizeof h) != 0)
        return fail(RT_E_INVALID, "the saved state belongs to a problem of another shape, bin count, angle set, "
                                  "precision, interpolation or periodic axes");
    if (bytes < (size_t)h.bytes) return fail(RT_E_INVALID, "src holds %zu bytes, the state needs %lld", bytes,
                                             (long long)h.bytes);
    const unsigned char *in = static_cast<const unsigned char *>(src);
    size_t off = pad256(sizeof h);
    for (auto &b : state_buffers(p)) {
        HIP_TRY(hipMemcpy(b.first, in + off, b.second, hipMemcpyDefault));
        off += pad256(b.second);
    }
    p->cold = cold;
    return RT_OK;
}

rt_status rt_formal_solve(rt_problem *p, const void *S_usr, void *J_usr, void *lambda_star, void *stream)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    if (!S_usr || !J_usr) return fail(RT_E_INVALID, "S and J are required");
    if (!p->have_fields) return fail(RT_E_INVALID, "rt_problem_set_fields has not been called");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nc = p->cells * p->nf;
    const double *S = static_cast<const double *>(S_usr);
    double *J = static_cast<double *>(J_usr);
    if (p->usr32) {
        HIP_TRY(launch_convert_f64(static_cast<const float *>(S_usr), p->stS, nc, st));
        S = p->stS;
        J = p->stJ;
    }
    HIP_TRY(hipMemsetAsync(p->frozen, 0, sizeof(int) * p->nf, st));
    rt_status s = collect_timing(p);
    if (s != RT_OK) return s;
    // the persistent schedule's dependency waits are bounded: one that ran out is
    // reported here, which needs a synchronisation (not possible under stream capture)
    bool check_waits = false;
    if (p->persistent) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(hipStreamIsCapturing(st, &cs));
        check_waits = cs == hipStreamCaptureStatusNone;
        if (check_waits) HIP_TRY(hipMemsetAsync(p->flags + 2, 0, sizeof(int), st));
    }
    s = sweep_current_S(p, S, st, true, p->nf);
    if (s != RT_OK) return s;
    if (check_waits) {
        HIP_TRY(hipMemcpyAsync(p->h_flags + 2, p->flags + 2, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (p->h_flags[2]) return fail(RT_E_HIP, "persistent sweep: a tile dependency wait ran out");
    }
    if (p->f32)
        HIP_TRY(launch_partial_sum<float>(static_cast<float *>(p->part), p->npart, S, 1, p->nf, p->cells, nullptr, J,
                                          st));
    else
        HIP_TRY(launch_partial_sum<double>(static_cast<double *>(p->part), p->npart, S, 0, p->nf, p->cells, nullptr,
                                           J, st));
    HIP_TRY(launch_flip_parity(p->parity, p->frozen, 0, p->nf, st));
    if (p->usr32) {
        HIP_TRY(launch_convert_f32(p->stJ, static_cast<float *>(J_usr), nc, st));
        if (lambda_star) HIP_TRY(launch_convert_f32(p->lam, static_cast<float *>(lambda_star), nc, st));
    } else if (lambda_star) {
        HIP_TRY(hipMemcpyAsync(lambda_star, p->lam, sizeof(double) * nc, hipMemcpyDeviceToDevice, st));
    }
    return RT_OK;
}

}  // extern "C"

namespace {

// Gauss-Seidel state of a problem: the rays going down (those crossing an x or y face
// first ahead of those crossing a z face first), their plane buffers and partial sums.
rt_status gs_prepare(rt_problem *p)
{
    if (p->gs_planes) return RT_OK;
    std::vector<int> down, steep;
    for (int k = 0; k < p->na; ++k) {
        if (!(p->rays[k].oct & 4)) continue;
        (p->rays[k].d == 2 ? steep : down).push_back(k);
    }
    const int ns = (int)down.size();
    down.insert(down.end(), steep.begin(), steep.end());
    const int nd = (int)down.size();
    const size_t rs = p->f32 ? sizeof(float) : sizeof(double);
    const size_t pxy = (size_t)p->n[0] * p->n[1];
    unsigned char *planes = nullptr, *part = nullptr, *chi_t = nullptr;
    double *S_t = nullptr;
    int *d_down = nullptr;
    rt_status s = dalloc(p, &planes, (size_t)p->nf * std::max(nd, 1) * 2 * pxy * rs);
    if (s == RT_OK) s = dalloc(p, &part, (size_t)std::max(nd, 1) * p->nf * pxy * rs);
    if (s == RT_OK) s = dalloc(p, &chi_t, (size_t)p->nf * p->cells * rs);
    if (s == RT_OK) s = dalloc(p, &S_t, (size_t)p->nf * p->cells);
    unsigned char *coef = nullptr, *gh = nullptr;
    const size_t nmax = (size_t)std::max(p->n[0], p->n[1]);
    if (s == RT_OK) s = dalloc(p, &coef, (size_t)p->nf * std::max(ns, 1) * 4 * pxy * rs);
    if (s == RT_OK) s = dalloc(p, &gh, (size_t)p->nf * std::max(ns, 1) * 4 * nmax * rs);
    double *ghS = nullptr;
    if (s == RT_OK) s = dalloc(p, &ghS, (size_t)p->nf * std::max(ns, 1) * 2 * nmax);
    if (s == RT_OK) s = dalloc(p, &d_down, (size_t)std::max(nd, 1));
    if (s != RT_OK) return s;
    if (nd > 0) HIP_TRY(hipMemcpy(d_down, down.data(), sizeof(int) * nd, hipMemcpyHostToDevice));
    p->gs_planes = planes;
    p->gs_part = part;
    p->gs_chi_t = chi_t;
    p->gs_coef = coef;
    p->gs_gh = gh;
    p->gs_ghS = ghS;
    p->gs_S_t = S_t;
    p->d_gs_down = d_down;
    p->gs_nd = nd;
    p->gs_ns = ns;
    return RT_OK;
}

template <typename Real>
GsArgs<Real> gs_args(rt_problem *p, double *S, double *J)
{
    GsArgs<Real> A{};
    for (int q = 0; q < 3; ++q) {
        A.n[q] = p->n[q];
        A.periodic[q] = p->periodic[q];
        A.bc_lo[q] = p->desc.bc_lo[q];
        A.bc_hi[q] = p->desc.bc_hi[q];
        A.wrap[q] = p->wrap[q];
    }
    A.nf = p->nf;
    A.na = p->na;
    A.cells = p->cells;
    A.pxy = (int64_t)p->n[0] * p->n[1];
    A.rays = p->d_rays;
    A.down = p->d_gs_down;
    A.nd = p->gs_nd;
    A.ns = p->gs_ns;
    if constexpr (sizeof(Real) == 4)
        A.chi = p->chi32;
    else
        A.chi = p->chi64;
    A.S = S;
    A.chi_t = static_cast<const Real *>(p->gs_chi_t);
    A.S_t = p->gs_S_t;
    A.B = p->B;
    A.eps = p->eps;
    A.lam = p->lam;
    for (int k = 0; k < 6; ++k) A.fixed[k] = p->desc.I_fixed[k];
    A.planes = static_cast<Real *>(p->gs_planes);
    A.part = static_cast<Real *>(p->gs_part);
    A.part_up = static_cast<const Real *>(p->part);
    A.J = J;
    A.frozen = p->frozen;
    A.parity = p->parity;
    A.blockmax = p->blockmax;
    A.nblk = kUpdateBlocks;
    A.tiles_x = (p->n[0] + kGsTile - 1) / kGsTile;
    A.ntiles = A.tiles_x * ((p->n[1] + kGsTile - 1) / kGsTile);
    A.coef = static_cast<Real *>(p->gs_coef);
    A.gh = static_cast<Real *>(p->gs_gh);
    A.ghS = p->gs_ghS;
    A.nmax = std::max(p->n[0], p->n[1]);
    A.steep_blocks = ((A.nd - A.ns) * A.ntiles + 7) / 8 * 8;
    return A;
}

// One Gauss-Seidel iteration: the rays going up over the whole grid with the old S
// (octants 0 .. 3 of the tile wavefront), then the rays going down plane by plane from
// the top with each plane's update as soon as its J is complete.
template <typename Real>
rt_status gs_iteration(rt_problem *p, double *S, double *J, hipStream_t st, bool timed, int active_bins)
{
    HIP_TRY(launch_gs_clear(p->blockmax, (int64_t)p->nf * kUpdateBlocks, st));
    SweepArgs<Real> U = sweep_args<Real>(p, S);
    U.noct = 4;
    if (p->cold) {
        HIP_TRY(launch_periodic_cold<Real>(U, st));
        p->cold = false;
    }
    HIP_TRY(launch_ghost_fill<Real>(U, st));
    // a profiled iteration also times the upward sweep's stage launches
    const bool tu = timed && p->prof && !p->prof_pending;
    for (int s = 0; s < p->nstages; ++s) {
        U.stage_off = p->stage_off[s];
        U.stage_cnt = p->stage_off[s + 1] - p->stage_off[s];
        U.stage = s;
        if (tu && s == 0) HIP_TRY(hipEventRecord(p->ev[0], st));
        if constexpr (sizeof(Real) == 8)
            HIP_TRY(launch_sweep_stage_f64(U, p->waves, 1, st));
        else
            HIP_TRY(launch_sweep_stage_f32(U, p->waves, 1, st));
        if (tu && s == p->nstages - 1) HIP_TRY(hipEventRecord(p->ev[1], st));
    }
    if (tu) {
        p->prof_pending = true;
        p->prof_pending_updates = (double)p->cells * (p->na / 2) * active_bins;   // octants 0 .. 3
    }
    const GsArgs<Real> A = gs_args<Real>(p, S, J);
    const int nz = p->n[2];
    // launch nz recomputes plane 0 only for the periodic memory of the in-plane axes
    const int last = (p->periodic[0] || p->periodic[1]) ? nz : nz - 1;
    timed = timed && p->prof && !p->gs_prof_pending && nz > 1 && p->gs_ns > 0;
    if (timed && p->gs_ev.empty()) {
        p->gs_ev.resize(2 * (size_t)nz);
        for (auto &e : p->gs_ev) HIP_TRY(hipEventCreate(&e));
    }
    for (int t = 0; t <= last; ++t) {
        const bool tt = timed && t >= 1 && t < nz;
        HIP_TRY(launch_gs_plane<Real>(A, t, st, tt ? p->gs_ev[2 * t] : nullptr, tt ? p->gs_ev[2 * t + 1] : nullptr));
        if (t < nz) HIP_TRY(launch_gs_update<Real>(A, nz - 1 - t, st));
    }
    if (timed) {
        p->gs_prof_pending = true;
        p->gs_pending_updates = (double)(nz - 1) * p->gs_ns * (double)p->n[0] * p->n[1] * active_bins;
    }
    return RT_OK;
}

rt_status ali_run(rt_problem *p, const rt_ali_opts *opts, double *S_inout, double *J_out, rt_ali_stats *stats,
                  hipStream_t st, std::chrono::steady_clock::time_point t0, bool gs);

// The executable graph of a chunk of k iterations with these arguments: cached, or
// captured from `body` on the problem's capture stream.  Capture always ends, also
// when the body fails.
template <typename Body>
rt_status chunk_graph(rt_problem *p, int k, bool gs, const double *S, const double *J, double delta_c,
                      int per_bin_stop, int fixed, Body body, hipGraphExec_t *out)
{
    for (auto &g : p->graphs)
        if (g.k == k && g.gs == gs && g.S == S && g.J == J && g.delta_c == delta_c && g.per_bin_stop == per_bin_stop &&
            g.fixed == fixed) {
            *out = g.exec;
            return RT_OK;
        }
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const rt_status s = body(p->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (s != RT_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return s != RT_OK ? s : fail(RT_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return fail(RT_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    if (p->graphs.size() >= 2) {
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        (void)hipGraphDestroy(p->graphs.front().graph);
        p->graphs.erase(p->graphs.begin());
    }
    rt_problem::GraphEntry g;
    g.k = k;
    g.gs = gs;
    g.S = S;
    g.J = J;
    g.delta_c = delta_c;
    g.per_bin_stop = per_bin_stop;
    g.fixed = fixed;
    g.graph = graph;
    g.exec = exec;
    p->graphs.push_back(g);
    *out = exec;
    return RT_OK;
}

// An ALI solve on the caller's S and J, or, for FP32 caller arrays, on the problem's
// FP64 copies of them: widened before (as far as the start values read them) and
// rounded back after.
rt_status ali_user(rt_problem *p, const rt_ali_opts *opts, void *S_usr, void *J_usr, rt_ali_stats *stats,
                   hipStream_t st, std::chrono::steady_clock::time_point t0, bool gs)
{
    if (!p->usr32)
        return ali_run(p, opts, static_cast<double *>(S_usr), static_cast<double *>(J_usr), stats, st, t0, gs);
    const int64_t nc = p->cells * p->nf;
    if (opts->warm_start == 1) HIP_TRY(launch_convert_f64(static_cast<const float *>(S_usr), p->stS, nc, st));
    if (opts->warm_start == 2) HIP_TRY(launch_convert_f64(static_cast<const float *>(J_usr), p->stJ, nc, st));
    const rt_status s = ali_run(p, opts, p->stS, p->stJ, stats, st, t0, gs);
    if (s == RT_OK || s == RT_NOT_CONVERGED || s == RT_E_NONFINITE) {
        HIP_TRY(launch_convert_f32(p->stS, static_cast<float *>(S_usr), nc, st));
        HIP_TRY(launch_convert_f32(p->stJ, static_cast<float *>(J_usr), nc, st));
    }
    return s;
}

}  // namespace

extern "C" {

rt_status rt_ali_solve(rt_problem *p, const rt_ali_opts *opts, void *S_inout, void *J_out, rt_ali_stats *stats,
                       void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!p || !opts) return fail(RT_E_INVALID, "problem and opts are required");
    CallScope scope(p->ctx, p->device);
    if (!S_inout || !J_out) return fail(RT_E_INVALID, "S_inout and J_out are required");
    if (!p->have_fields) return fail(RT_E_INVALID, "rt_problem_set_fields has not been called");
    {
        rt_status so = check_ali_opts(opts);
        if (so != RT_OK) return so;
    }
    return ali_user(p, opts, S_inout, J_out, stats, static_cast<hipStream_t>(stream), t0, false);
}

rt_status rt_ali_solve_gs(rt_problem *p, const rt_ali_opts *opts, void *S_inout, void *J_out,
                          rt_ali_stats *stats, void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!p || !opts) return fail(RT_E_INVALID, "problem and opts are required");
    CallScope scope(p->ctx, p->device);
    if (!S_inout || !J_out) return fail(RT_E_INVALID, "S_inout and J_out are required");
    if (!p->have_fields) return fail(RT_E_INVALID, "rt_problem_set_fields has not been called");
    {
        rt_status so = check_ali_opts(opts);
        if (so != RT_OK) return so;
    }
    if (p->desc.order != RT_SC_LINEAR || p->plane_order)
        return fail(RT_E_UNSUPPORTED, "Gauss-Seidel needs first-order segments and bilinear upwind intensities");
    if (p->periodic[2]) return fail(RT_E_UNSUPPORTED, "Gauss-Seidel orders the planes along z, which must not be periodic");
    if (p->persistent) return fail(RT_E_UNSUPPORTED, "Gauss-Seidel runs with the staged sweep schedule");
    if (p->n[0] > kGsMaxLanes || p->n[1] > kGsMaxLanes)
        return fail(RT_E_UNSUPPORTED, "Gauss-Seidel needs nx and ny <= %d", kGsMaxLanes);
    if (p->na / 2 > kGsMaxDown) return fail(RT_E_UNSUPPORTED, "Gauss-Seidel takes at most %d rays", 2 * kGsMaxDown);
    rt_status s = gs_prepare(p);
    if (s != RT_OK) return s;
    return ali_user(p, opts, S_inout, J_out, stats, static_cast<hipStream_t>(stream), t0, true);
}

}  // extern "C"

namespace {

rt_status ali_run(rt_problem *p, const rt_ali_opts *opts, double *S_inout, double *J_out, rt_ali_stats *stats,
                  hipStream_t st, std::chrono::steady_clock::time_point t0, bool gs)
{
    {
        rt_status s0 = ali_start(p, opts, S_inout, J_out, st);
        if (s0 != RT_OK) return s0;
    }
    if (gs) {
        // y-fastest copies of chi and of the start S for the chains along x
        if (p->f32)
            HIP_TRY(launch_gs_transpose<float>(p->chi32, static_cast<float *>(p->gs_chi_t), p->nf, p->n, st));
        else
            HIP_TRY(launch_gs_transpose<double>(p->chi64, static_cast<double *>(p->gs_chi_t), p->nf, p->n, st));
        HIP_TRY(launch_gs_transpose<double>(S_inout, p->gs_S_t, p->nf, p->n, st));
    }

    const bool fixed = opts->fixed_iters > 0;
    const int total = fixed ? opts->fixed_iters : opts->max_iter;
    const int every = opts->check_every > 0 ? opts->check_every : 16;
    AliCtl ctl = ctl_of(p);
    int done = 0;
    bool nonfinite = false;
    int active = p->nf;
    {
        rt_status s = collect_timing(p);
        if (s != RT_OK) return s;
    }
    // k iterations on stream cs; the first one's sweep is timed when profiling is on
    auto chunk = [&](int k, hipStream_t cs) -> rt_status {
        for (int j = 0; j < k; ++j) {
            if (gs) {
                rt_status s = p->f32 ? gs_iteration<float>(p, S_inout, J_out, cs, j == 0, active)
                                     : gs_iteration<double>(p, S_inout, J_out, cs, j == 0, active);
                if (s != RT_OK) return s;
                HIP_TRY(launch_ali_finalize(ctl, p->nf, opts->delta_c, opts->per_bin_stop ? 1 : 0, fixed ? 1 : 0, cs));
                continue;
            }
            rt_status s = sweep_current_S(p, S_inout, cs, j == 0, active);
            if (s != RT_OK) return s;
            if (p->f32)
                HIP_TRY(launch_ali_update<float>(static_cast<float *>(p->part), p->npart, 1, p->nf, p->cells, p->B,
                                                 p->eps, p->lam, S_inout, J_out, ctl, cs));
            else
                HIP_TRY(launch_ali_update<double>(static_cast<double *>(p->part), p->npart, 0, p->nf, p->cells, p->B,
                                                  p->eps, p->lam, S_inout, J_out, ctl, cs));
            HIP_TRY(launch_ali_finalize(ctl, p->nf, opts->delta_c, opts->per_bin_stop ? 1 : 0, fixed ? 1 : 0, cs));
        }
        return RT_OK;
    };
    // Chunks run as captured graphs (the same launches with the same arguments every
    // chunk; frozen bins make their kernels return at once), except while the sweep
    // is being timed.  The one-time periodic initialisation runs before, eagerly.
    const bool use_graph = p->use_graphs && !p->prof;
    if (use_graph && p->cold) {
        if (p->plane_order) {
            if (p->f32)
                HIP_TRY(launch_plane_cold<float>(plane_args<float>(p, S_inout), st));
            else
                HIP_TRY(launch_plane_cold<double>(plane_args<double>(p, S_inout), st));
        } else {
            if (p->f32)
                HIP_TRY(launch_periodic_cold<float>(sweep_args<float>(p, S_inout), st));
            else
                HIP_TRY(launch_periodic_cold<double>(sweep_args<double>(p, S_inout), st));
        }
        p->cold = false;
    }
    for (int it = 0; it < total && !done;) {
        const int k = std::min(every, total - it);
        if (use_graph) {
            hipGraphExec_t ex = nullptr;
            rt_status s = chunk_graph(p, k, gs, S_inout, J_out, opts->delta_c, opts->per_bin_stop ? 1 : 0,
                                      fixed ? 1 : 0, [&](hipStream_t cs) { return chunk(k, cs); }, &ex);
            if (s != RT_OK) return s;
            HIP_TRY(hipGraphLaunch(ex, st));
        } else {
            rt_status s = chunk(k, st);
            if (s != RT_OK) return s;
        }
        it += k;
        HIP_TRY(hipMemcpyAsync(p->h_flags, p->flags, sizeof(int) * 3, hipMemcpyDeviceToHost, st));
        if (p->prof) HIP_TRY(hipMemcpyAsync(p->h_frozen, p->frozen, sizeof(int) * p->nf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        done = p->h_flags[0];
        nonfinite = p->h_flags[1] != 0;
        if (p->h_flags[2]) return fail(RT_E_HIP, "persistent sweep: a tile dependency wait ran out");
        {
            rt_status s = collect_timing(p);
            if (s != RT_OK) return s;
        }
        if (p->prof) {
            active = 0;
            for (int f = 0; f < p->nf; ++f) active += p->h_frozen[f] == 0;
        }
    }
    std::vector<int> iters(p->nf);
    std::vector<double> resid(p->nf);
    HIP_TRY(hipMemcpyAsync(iters.data(), p->iters, sizeof(int) * p->nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(resid.data(), p->resid, sizeof(double) * p->nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int conv = 0, maxit = 0;
    double maxr = 0.0;
    for (int f = 0; f < p->nf; ++f) {
        conv += resid[f] <= opts->delta_c;
        maxit = std::max(maxit, iters[f]);
        maxr = std::max(maxr, resid[f]);
    }
    if (stats) {
        stats->iterations = maxit;
        stats->bins_converged = conv;
        stats->max_rel_dS = maxr;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (nonfinite) return fail(RT_E_NONFINITE, "non-finite residual during the Lambda iteration");
    if (!fixed && conv < p->nf) return RT_NOT_CONVERGED;
    return RT_OK;
}

}  // namespace

extern "C" {

namespace {
void drop_graphs(rt_problem *p)
{
    for (auto &g : p->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
}
}  // namespace

rt_status rt_problem_set_waves(rt_problem *p, int32_t waves)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    if (p->plane_order) return fail(RT_E_UNSUPPORTED, "the plane-ordered sweep has no wave count");
    const int wmax = std::min(p->R, kMaxWaves);
    if (waves < 1 || waves > wmax) return fail(RT_E_INVALID, "waves must be in [1, %d]", wmax);
    if (sweep_lds_bytes(p->f32 ? 4 : 8, waves, 1, p->R > waves, p->desc.order) > p->lds_limit)
        return fail(RT_E_UNSUPPORTED, "%d waves need more LDS than the device allows", (int)waves);
    if (waves != p->waves) drop_graphs(p);   // captured launches carry the old shape
    p->waves = waves;
    if (p->persistent) persistent_grid(p);
    return RT_OK;
}

rt_status rt_problem_set_wait_limit(rt_problem *p, double microseconds)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    if (!(microseconds >= 0.0) || microseconds > 1e9) return fail(RT_E_INVALID, "wait limit must be in [0, 1e9] us");
    const uint64_t ticks = (uint64_t)(microseconds * 1e-3 * (double)p->wall_khz);
    if (ticks != p->wait_ticks) drop_graphs(p);   // captured launches carry the old bound
    p->wait_ticks = ticks;
    return RT_OK;
}

rt_status rt_problem_tune(rt_problem *p, const void *S_usr, int32_t reps, int32_t *waves_out, float *ms_out,
                          void *stream)
{
    if (!p || !S_usr || !waves_out) return fail(RT_E_INVALID, "problem, S and waves_out are required");
    CallScope scope(p->ctx, p->device);
    if (!p->have_fields) return fail(RT_E_INVALID, "rt_problem_set_fields has not been called");
    if (p->plane_order) return fail(RT_E_UNSUPPORTED, "the plane-ordered sweep has no wave count");
    if (reps < 1) return fail(RT_E_INVALID, "reps must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double *S = static_cast<const double *>(S_usr);
    if (p->usr32) {
        HIP_TRY(launch_convert_f64(static_cast<const float *>(S_usr), p->stS, p->cells * p->nf, st));
        S = p->stS;
    }
    const int wmax = std::min(p->R, kMaxWaves);
    const bool cold = p->cold;
    const int keep = p->waves;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(RT_E_HIP, "hipEventCreate: %s", hipGetErrorString(he));
    }
    rt_status s = RT_OK;
    int best = keep;
    float best_ms = 0.0f;
    he = hipMemsetAsync(p->frozen, 0, sizeof(int) * p->nf, st);
    for (int w = 1; w <= wmax && s == RT_OK && he == hipSuccess; ++w) {
        if (ms_out) ms_out[w - 1] = -1.0f;
        if (sweep_lds_bytes(p->f32 ? 4 : 8, w, 1, p->R > w, p->desc.order) > p->lds_limit) continue;
        p->waves = w;
        if (p->persistent) persistent_grid(p);
        s = sweep_current_S(p, S, st);   // untimed: caches warm, cold memory filled
        if (s == RT_OK) he = hipEventRecord(e0, st);
        for (int r = 0; r < reps && s == RT_OK && he == hipSuccess; ++r) s = sweep_current_S(p, S, st);
        if (s == RT_OK && he == hipSuccess) he = hipEventRecord(e1, st);
        if (s == RT_OK && he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (s == RT_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (s != RT_OK || he != hipSuccess) break;
        ms /= (float)reps;
        if (ms_out) ms_out[w - 1] = ms;
        if (best_ms == 0.0f || ms < best_ms) {
            best_ms = ms;
            best = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the sweeps wrote only the periodic slot the next sweep overwrites; a cold problem
    // stays cold (its next solve fills the memory from its own S)
    p->cold = cold;
    if (best != keep) drop_graphs(p);
    p->waves = best;
    if (p->persistent) persistent_grid(p);
    if (s != RT_OK) return s;
    if (he != hipSuccess) {
        (void)hipGetLastError();
        return fail(RT_E_HIP, "timing the sweep failed: %s", hipGetErrorString(he));
    }
    *waves_out = best;
    return RT_OK;
}

rt_status rt_problem_use_graphs(rt_problem *p, int32_t enable)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    p->use_graphs = enable != 0;
    return RT_OK;
}

rt_status rt_ali_bin_stats(rt_problem *p, int32_t *iters, double *resid, void *stream)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (iters) HIP_TRY(hipMemcpyAsync(iters, p->iters, sizeof(int) * p->nf, hipMemcpyDeviceToHost, st));
    if (resid) HIP_TRY(hipMemcpyAsync(resid, p->resid, sizeof(double) * p->nf, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return RT_OK;
}

rt_status rt_problem_profile(rt_problem *p, int32_t enable)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    rt_status s = collect_timing(p);
    if (s != RT_OK) return s;
    if (enable && p->ev.empty()) {
        p->ev.resize(2);
        for (auto &e : p->ev) HIP_TRY(hipEventCreate(&e));
    }
    p->prof = enable != 0;
    p->prof_ms = p->prof_updates = 0.0;
    p->prof_launches = p->prof_sweeps = 0;
    p->gs_prof_ms = p->gs_prof_updates = 0.0;
    p->gs_prof_launches = 0;
    return RT_OK;
}

rt_status rt_problem_profile_read(rt_problem *p, rt_profile *out)
{
    if (!p || !out) return fail(RT_E_INVALID, "problem and out are required");
    CallScope scope(p->ctx, p->device);
    rt_status s = collect_timing(p);
    if (s != RT_OK) return s;
    out->kernel_ms = p->prof_ms;
    out->launches = p->prof_launches;
    out->sweeps = p->prof_sweeps;
    out->updates = p->prof_updates;
    out->stages = p->nstages;
    out->chain_ms = p->gs_prof_ms;
    out->chain_launches = p->gs_prof_launches;
    out->chain_updates = p->gs_prof_updates;
    return RT_OK;
}

}  // extern "C"

namespace {

// Outputs of the moments epilogue in FP64 (the caller's arrays, or the problem's FP64
// staging of FP32 caller arrays).
struct MomOut64 {
    double *J, *H, *K, *J_int, *H_int, *K_int, *f_int, *Q_int;
    double *heating;
};

rt_status moments_core(rt_problem *p, const double *S, const MomOut64 &out, hipStream_t st)
{
    const bool want_int = out.J_int || out.H_int || out.K_int || out.f_int || out.Q_int || out.heating;
    if (!(out.J || out.H || out.K || want_int)) return RT_OK;
    const int64_t cells = p->cells;
    const size_t rs = p->f32 ? sizeof(float) : sizeof(double);

    // scratch: bins are processed in chunks so the moment partials fit (per octant, or
    // per class of the plane-ordered sweep)
    if (!p->mom_part) {
        const size_t per_bin = (size_t)cells * ((size_t)p->npart * 10 * rs + 11 * sizeof(double));
        const size_t budget = (size_t)4 << 30;
        p->mom_nfc = (int)std::max<size_t>(1, std::min<size_t>((size_t)p->nf, budget / std::max<size_t>(per_bin, 1)));
        rt_status a;
        unsigned char *pb = nullptr;
        if ((a = dalloc(p, &pb, (size_t)p->npart * 10 * p->mom_nfc * cells * rs)) != RT_OK) return a;
        p->mom_part = pb;
        if ((a = dalloc(p, &p->mom_tmp, (size_t)10 * p->mom_nfc * cells)) != RT_OK) return a;
        if ((a = dalloc(p, &p->mom_q, (size_t)p->mom_nfc * cells)) != RT_OK) return a;
        if ((a = dalloc(p, &p->mom_qint, (size_t)cells)) != RT_OK) return a;
        if ((a = dalloc(p, &p->mom_wnu, (size_t)p->nf)) != RT_OK) return a;
        if ((a = dalloc(p, &p->mom_sum, (size_t)1025)) != RT_OK) return a;
        if (hipHostMalloc((void **)&p->h_sum, sizeof(double), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            p->h_sum = nullptr;
            return fail(RT_E_OOM, "pinned host allocation failed");
        }
        HIP_TRY(hipMemcpy(p->mom_wnu, p->w_nu.data(), sizeof(double) * p->nf, hipMemcpyHostToDevice));
    }
    MomConst mc{};
    mc.m[0] = 1.0;
    for (const RayGeo &g : p->rays) {
        const double *m = g.mu;
        mc.m[1] += g.wk * m[0];
        mc.m[2] += g.wk * m[1];
        mc.m[3] += g.wk * m[2];
        mc.m[4] += g.wk * m[0] * m[0];
        mc.m[5] += g.wk * m[1] * m[1];
        mc.m[6] += g.wk * m[2] * m[2];
        mc.m[7] += g.wk * m[0] * m[1];
        mc.m[8] += g.wk * m[0] * m[2];
        mc.m[9] += g.wk * m[1] * m[2];
    }
    const double h[3] = {p->desc.dx, p->desc.dy, p->desc.dz};
    double *Qint = out.Q_int ? out.Q_int : (out.heating ? p->mom_qint : nullptr);
    HIP_TRY(hipMemsetAsync(p->frozen, 0, sizeof(int) * p->nf, st));
    for (int f0 = 0; f0 < p->nf; f0 += p->mom_nfc) {
        const int cnt = std::min(p->mom_nfc, p->nf - f0);
        SweepMode mode;
        mode.nq = 10;
        mode.f0 = f0;
        mode.nfc = cnt;
        mode.part = p->mom_part;
        // one ray per wave: the partial sums come from the waves' cubes and the
        // LDS is that of the J sweep; otherwise one wave with ten accumulated tiles
        mode.waves = p->R <= p->waves ? p->waves : 1;
        rt_status s = p->f32 ? run_sweep<float>(p, S, st, false, 0, mode) : run_sweep<double>(p, S, st, false, 0, mode);
        if (s != RT_OK) return s;
        HIP_TRY(launch_flip_parity(p->parity, p->frozen, f0, cnt, st));
        if (p->f32)
            HIP_TRY(launch_moments_combine<float>(static_cast<float *>(p->mom_part), p->npart, S, 1, f0, cnt, p->nf,
                                                  cells, mc, out.J, out.H, out.K, p->mom_tmp, st));
        else
            HIP_TRY(launch_moments_combine<double>(static_cast<double *>(p->mom_part), p->npart, S, 0, f0, cnt, p->nf,
                                                   cells, mc, out.J, out.H, out.K, p->mom_tmp, st));
        if (Qint) HIP_TRY(launch_moments_q(p->mom_tmp, f0, cnt, p->n, h, p->periodic, p->chi64, p->eps, p->B, p->mom_q, st));
        if (want_int) {
            const bool needK = out.K_int || out.f_int;
            double *Jt = (out.J_int || out.f_int) ? out.J_int : nullptr;
            HIP_TRY(launch_moments_integrate(p->mom_tmp, p->mom_q, p->mom_wnu, f0, cnt, cells, f0 == 0, Jt, out.H_int,
                                             needK ? out.K_int : nullptr, Qint, st));
        }
    }
    if (out.f_int) {
        if (!out.J_int || !out.K_int) return fail(RT_E_INVALID, "f_int needs J_int and K_int buffers");
        HIP_TRY(launch_eddington(out.J_int, out.K_int, cells, out.f_int, st));
    }
    if (out.heating) {
        const int nblk = (int)std::min<int64_t>(1024, (cells + 255) / 256);
        HIP_TRY(launch_sum(Qint, cells, h[0] * h[1] * h[2], p->mom_sum, nblk, p->mom_sum + 1024, st));
        HIP_TRY(hipMemcpyAsync(p->h_sum, p->mom_sum + 1024, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *out.heating = *p->h_sum;
    }
    return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_moments(rt_problem *p, const void *S_usr, const rt_moments_out *out, void *stream)
{
    if (!p) return fail(RT_E_INVALID, "problem is NULL");
    CallScope scope(p->ctx, p->device);
    if (!S_usr || !out) return fail(RT_E_INVALID, "S and out are required");
    if (!p->have_fields) return fail(RT_E_INVALID, "rt_problem_set_fields has not been called");
    if (out->f_int && (!out->J_int || !out->K_int)) return fail(RT_E_INVALID, "f_int needs J_int and K_int buffers");
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *const user[8] = {out->J, out->H, out->K, out->J_int, out->H_int, out->K_int, out->f_int, out->Q_int};
    if (!p->usr32) {
        MomOut64 o{};
        double **f64[8] = {&o.J, &o.H, &o.K, &o.J_int, &o.H_int, &o.K_int, &o.f_int, &o.Q_int};
        for (int k = 0; k < 8; ++k) *f64[k] = static_cast<double *>(user[k]);
        o.heating = out->heating;
        return moments_core(p, static_cast<const double *>(S_usr), o, st);
    }
    // FP32 caller arrays: S widened, every requested output computed into FP64 staging
    // (allocated on first use) and rounded into the caller's array
    const int64_t nc = p->cells * p->nf, c = p->cells;
    const int64_t count[8] = {nc, 3 * nc, 6 * nc, c, 3 * c, 6 * c, 6 * c, c};
    MomOut64 o{};
    double **f64[8] = {&o.J, &o.H, &o.K, &o.J_int, &o.H_int, &o.K_int, &o.f_int, &o.Q_int};
    for (int k = 0; k < 8; ++k) {
        if (!user[k]) continue;
        if (!p->mst[k]) {
            rt_status a = dalloc(p, &p->mst[k], (size_t)count[k]);
            if (a != RT_OK) return a;
        }
        *f64[k] = p->mst[k];
    }
    o.heating = out->heating;
    HIP_TRY(launch_convert_f64(static_cast<const float *>(S_usr), p->stS, nc, st));
    rt_status s = moments_core(p, p->stS, o, st);
    if (s != RT_OK) return s;
    for (int k = 0; k < 8; ++k)
        if (user[k]) HIP_TRY(launch_convert_f32(p->mst[k], static_cast<float *>(user[k]), count[k], st));
    return RT_OK;
}

rt_status rt_ali_solve_batch(rt_context *ctx, rt_problem *const *problems, int32_t n, const rt_ali_opts *opts,
                             void *const *S_inout, void *const *J_out, rt_ali_stats *stats, rt_status *results,
                             void *stream)
{
    auto t0 = std::chrono::steady_clock::now();
    CallScope scope(ctx, ctx ? ctx->device : -1);
    if (!problems || !opts || !S_inout || !J_out) return fail(RT_E_INVALID, "problems, opts, S_inout and J_out are required");
    if (n < 1) return fail(RT_E_INVALID, "n must be >= 1");
    {
        rt_status so = check_ali_opts(opts);
        if (so != RT_OK) return so;
    }
    for (int i = 0; i < n; ++i) {
        rt_problem *p = problems[i];
        if (!p) return fail(RT_E_INVALID, "problem %d is NULL", i);
        if (!S_inout[i] || !J_out[i]) return fail(RT_E_INVALID, "S_inout/J_out of problem %d missing", i);
        if (!p->have_fields) return fail(RT_E_INVALID, "problem %d: rt_problem_set_fields has not been called", i);
        for (int j = 0; j < i; ++j)
            if (problems[j] == p) return fail(RT_E_INVALID, "problem %d appears twice in the batch", i);
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i)
        if (problems[i]->device != dev)
            return fail(RT_E_INVALID, "problem %d lives on device %d, the batch runs on %d", i, problems[i]->device, dev);
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchRunner run(st);
    for (int i = 0; i < n; ++i) {
        rt_problem *p = problems[i];
        BatchItem it;
        it.p = p;
        if (p->usr32) {
            // FP64 copies of FP32 caller arrays, as far as the start values read them
            const int64_t nc = p->cells * p->nf;
            if (opts->warm_start == 1) HIP_TRY(launch_convert_f64(static_cast<const float *>(S_inout[i]), p->stS, nc, st));
            if (opts->warm_start == 2) HIP_TRY(launch_convert_f64(static_cast<const float *>(J_out[i]), p->stJ, nc, st));
            it.S = p->stS;
            it.J = p->stJ;
        } else {
            it.S = static_cast<double *>(S_inout[i]);
            it.J = static_cast<double *>(J_out[i]);
        }
        it.opts = *opts;
        it.total = opts->fixed_iters > 0 ? opts->fixed_iters : opts->max_iter;
        it.tag = (uint64_t)i;
        rt_status s = run.add(it);
        if (s != RT_OK) return s;
    }
    const int every = opts->fixed_iters > 0 ? opts->fixed_iters : (opts->check_every > 0 ? opts->check_every : 16);
    std::vector<BatchItem> finished;
    std::vector<double> secs(n, 0.0);
    std::vector<char> nonfin(n, 0);
    std::vector<rt_status> errs(n, RT_OK);
    while (run.size() > 0) {
        const size_t before = finished.size();
        rt_status s = run.chunk(every, finished);
        if (s != RT_OK) return s;
        const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (size_t k = before; k < finished.size(); ++k) {
            secs[finished[k].tag] = t;
            nonfin[finished[k].tag] = finished[k].nonfinite;
            errs[finished[k].tag] = finished[k].err;
        }
    }
    rt_status worst = RT_OK;
    for (int i = 0; i < n; ++i) {
        rt_problem *p = problems[i];
        if (p->usr32) {
            const int64_t nc = p->cells * p->nf;
            HIP_TRY(launch_convert_f32(p->stS, static_cast<float *>(S_inout[i]), nc, st));
            HIP_TRY(launch_convert_f32(p->stJ, static_cast<float *>(J_out[i]), nc, st));
        }
        rt_status r = RT_OK;
        rt_status s = ali_stats(p, opts, nonfin[i] != 0, secs[i], stats ? &stats[i] : nullptr, st, &r);
        if (s != RT_OK) return s;
        if (errs[i] != RT_OK) r = errs[i];
        if (results) results[i] = r;
        if (r == RT_E_HIP) worst = RT_E_HIP;
        else if (r == RT_E_NONFINITE && worst != RT_E_HIP) worst = RT_E_NONFINITE;
        else if (r == RT_NOT_CONVERGED && worst == RT_OK) worst = RT_NOT_CONVERGED;
    }
    if (worst == RT_E_HIP)
        return fail(RT_E_HIP, "persistent sweep: a tile dependency wait ran out in a problem of the batch");
    if (worst == RT_E_NONFINITE) return fail(RT_E_NONFINITE, "non-finite residual in at least one problem of the batch");
    return worst;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Serving loop (rt_server_*): a worker thread owns a stream and a BatchRunner; it
// admits queued requests at the batch's checks within the HBM budget, runs one check
// interval of the whole batch, and records the requests that finished.
// ---------------------------------------------------------------------------------
struct rt_server {
    struct Request {
        BatchItem item;
        void *S_usr = nullptr, *J_usr = nullptr;   // the caller's arrays (FP32 ones are widened)
        hipEvent_t ready = nullptr;                 // recorded on the caller's stream at submission
        size_t bytes = 0;
        std::chrono::steady_clock::time_point t_submit;
        bool done = false;
        rt_status result = RT_OK;
        rt_ali_stats stats{};
    };
    rt_context *ctx = nullptr;
    int device = 0;
    size_t budget = 0;
    int every = 16;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;              // waiting tickets, arrival order
    std::map<uint64_t, Request> reqs;        // every unreleased ticket
    size_t running_bytes = 0;
    int running = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool dead = false;                       // the worker has exited after a failure
    std::thread worker;

    void finish(uint64_t t, rt_status r, const rt_ali_stats &st)
    {
        Request &q = reqs[t];
        q.item.p->server_refs.fetch_sub(1);
        q.done = true;
        q.result = r;
        q.stats = st;
        q.stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - q.t_submit).count();
        running_bytes -= q.bytes;
        --running;
    }

    // a queued request that will never run: its submission event is no longer needed
    void abandon(uint64_t t, rt_status r)
    {
        Request &q = reqs[t];
        q.item.p->server_refs.fetch_sub(1);
        q.done = true;
        q.result = r;
        if (q.ready) (void)hipEventDestroy(q.ready);
        q.ready = nullptr;
    }

    void run()
    {
        t_ctx = ctx;
        (void)hipSetDevice(device);
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            std::lock_guard<std::mutex> lk(mu);
            dead = true;
            for (uint64_t t : queue) abandon(t, RT_E_HIP);
            queue.clear();
            cv.notify_all();
            return;
        }
        {
            BatchRunner batch(st);
            for (;;) {
                std::vector<uint64_t> admit;
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return stop || !queue.empty() || batch.size() > 0; });
                    if (stop && queue.empty() && batch.size() == 0) break;
                    while (!queue.empty()) {
                        Request &q = reqs[queue.front()];
                        if (running > 0 && running_bytes + q.bytes > budget) break;
                        admit.push_back(queue.front());
                        running_bytes += q.bytes;
                        ++running;
                        queue.pop_front();
                    }
                }
                for (uint64_t t : admit) {
                    BatchItem it;
                    hipEvent_t ready = nullptr;
                    void *S_usr = nullptr, *J_usr = nullptr;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        Request &q = reqs[t];
                        it = q.item;
                        ready = q.ready;
                        q.ready = nullptr;
                        S_usr = q.S_usr;
                        J_usr = q.J_usr;
                    }
                    // the caller's work on its stream before the submission comes first
                    rt_status s = RT_OK;
                    if (ready) {
                        if (hipStreamWaitEvent(st, ready, 0) != hipSuccess) s = fail(RT_E_HIP, "hipStreamWaitEvent failed");
                        (void)hipEventDestroy(ready);
                    }
                    rt_problem *p = it.p;
                    if (s == RT_OK && p->usr32) {
                        const int64_t nc = p->cells * p->nf;
                        hipError_t e = hipSuccess;
                        if (it.opts.warm_start == 1) e = launch_convert_f64(static_cast<const float *>(S_usr), p->stS, nc, st);
                        if (e == hipSuccess && it.opts.warm_start == 2)
                            e = launch_convert_f64(static_cast<const float *>(J_usr), p->stJ, nc, st);
                        if (e != hipSuccess) s = fail(RT_E_HIP, "conversion launch failed: %s", hipGetErrorString(e));
                    }
                    if (s == RT_OK) s = batch.add(it);
                    if (s != RT_OK) {
                        std::lock_guard<std::mutex> lk(mu);
                        finish(t, s, rt_ali_stats{});
                    }
                }
                if (batch.size() == 0) continue;
                std::vector<BatchItem> fin;
                rt_status s = batch.chunk(every, fin);
                if (s != RT_OK) {
                    // the stream or a launch failed: every running request ends with it
                    std::lock_guard<std::mutex> lk(mu);
                    for (const BatchItem &b : batch.items()) finish(b.tag, s, rt_ali_stats{});
                    for (const BatchItem &b : fin) finish(b.tag, s, rt_ali_stats{});
                    break;
                }
                for (const BatchItem &b : fin) {
                    rt_ali_stats sts{};
                    rt_status r = RT_OK;
                    rt_status s2 = RT_OK;
                    if (b.p->usr32) {
                        // round the FP64 copies into the caller's FP32 arrays (the
                        // synchronisation in ali_stats completes them before the request
                        // is reported finished)
                        void *S_usr = nullptr, *J_usr = nullptr;
                        {
                            std::lock_guard<std::mutex> lk(mu);
                            S_usr = reqs[b.tag].S_usr;
                            J_usr = reqs[b.tag].J_usr;
                        }
                        const int64_t nc = b.p->cells * b.p->nf;
                        hipError_t e = launch_convert_f32(b.p->stS, static_cast<float *>(S_usr), nc, st);
                        if (e == hipSuccess) e = launch_convert_f32(b.p->stJ, static_cast<float *>(J_usr), nc, st);
                        if (e != hipSuccess) s2 = fail(RT_E_HIP, "conversion launch failed: %s", hipGetErrorString(e));
                    }
                    if (s2 == RT_OK) s2 = ali_stats(b.p, &b.opts, b.nonfinite, 0.0, &sts, st, &r);
                    if (s2 == RT_OK && b.err != RT_OK) r = b.err;
                    std::lock_guard<std::mutex> lk(mu);
                    finish(b.tag, s2 != RT_OK ? s2 : r, sts);
                }
                cv.notify_all();
            }
        }
        {
            // anything still queued after a failure ends with that failure
            std::lock_guard<std::mutex> lk(mu);
            for (uint64_t t : queue) abandon(t, RT_E_HIP);
            queue.clear();
        }
        if (st) (void)hipStreamDestroy(st);
        {
            std::lock_guard<std::mutex> lk(mu);
            dead = true;
        }
        cv.notify_all();
    }
};

extern "C" {

rt_status rt_server_create(rt_context *ctx, size_t hbm_budget, int32_t check_every, rt_server **out)
{
    CallScope scope(ctx, ctx ? ctx->device : -1);
    if (!out) return fail(RT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (check_every < 0) return fail(RT_E_INVALID, "check_every must be >= 0");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    rt_server *srv = new rt_server();
    srv->ctx = ctx;
    srv->device = dev;
    srv->budget = hbm_budget;
    srv->every = check_every > 0 ? check_every : 16;
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return RT_OK;
}

rt_status rt_server_submit(rt_server *srv, rt_problem *p, const rt_ali_opts *opts, void *S_inout, void *J_out,
                           void *stream, uint64_t *ticket)
{
    if (!srv) return fail(RT_E_INVALID, "server is NULL");
    CallScope scope(srv->ctx, srv->device);
    if (!p || !opts || !S_inout || !J_out || !ticket)
        return fail(RT_E_INVALID, "server, problem, opts, S_inout, J_out and ticket are required");
    if (!p->have_fields) return fail(RT_E_INVALID, "rt_problem_set_fields has not been called");
    if (p->device != srv->device)
        return fail(RT_E_INVALID, "the problem lives on device %d, the server on %d", p->device, srv->device);
    {
        rt_status so = check_ali_opts(opts);
        if (so != RT_OK) return so;
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return fail(RT_E_INVALID, "server is shutting down");
        if (srv->dead) return fail(RT_E_HIP, "server worker stopped after a device failure");
        for (const auto &kv : srv->reqs)
            if (!kv.second.done && kv.second.item.p == p) return fail(RT_E_INVALID, "problem already has a pending request");
    }
    rt_server::Request q;
    q.item.p = p;
    q.item.S = p->usr32 ? p->stS : static_cast<double *>(S_inout);
    q.item.J = p->usr32 ? p->stJ : static_cast<double *>(J_out);
    q.S_usr = S_inout;
    q.J_usr = J_out;
    q.item.opts = *opts;
    q.item.total = opts->fixed_iters > 0 ? opts->fixed_iters : opts->max_iter;
    q.bytes = state_bytes(&p->desc, p->na);
    HIP_TRY(hipEventCreateWithFlags(&q.ready, hipEventDisableTiming));
    if (hipEventRecord(q.ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipEventDestroy(q.ready);
        return fail(RT_E_HIP, "hipEventRecord on the caller's stream failed");
    }
    q.t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    const uint64_t t = srv->next_ticket++;
    q.item.tag = t;
    srv->reqs[t] = q;
    p->server_refs.fetch_add(1);
    srv->queue.push_back(t);
    *ticket = t;
    srv->cv.notify_all();
    return RT_OK;
}

rt_status rt_server_poll(rt_server *srv, uint64_t ticket, rt_ali_stats *stats, rt_status *result)
{
    if (!srv) return fail(RT_E_INVALID, "server is NULL");
    CallScope scope(srv->ctx, -1);
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(RT_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) return RT_E_BUSY;
    if (stats) *stats = it->second.stats;
    if (result) *result = it->second.result;
    return RT_OK;
}

rt_status rt_server_release(rt_server *srv, uint64_t ticket)
{
    if (!srv) return fail(RT_E_INVALID, "server is NULL");
    CallScope scope(srv->ctx, -1);
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(RT_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done) return fail(RT_E_INVALID, "ticket %llu has not finished", (unsigned long long)ticket);
    srv->reqs.erase(it);
    return RT_OK;
}

rt_status rt_server_load(rt_server *srv, int32_t *queued, int32_t *running, size_t *running_bytes)
{
    if (!srv) return fail(RT_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (queued) *queued = (int32_t)srv->queue.size();
    if (running) *running = srv->running;
    if (running_bytes) *running_bytes = srv->running_bytes;
    return RT_OK;
}

rt_status rt_server_destroy(rt_server *srv)
{
    if (!srv) return RT_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    delete srv;
    return RT_OK;
}

}  // extern "C"

