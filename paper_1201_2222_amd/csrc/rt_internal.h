// Internal declarations shared by the host runtime (rt_api.cpp) and the HIP
// kernels (rt_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtsc {

enum { BC_VACUUM = 0, BC_THERMAL = 1, BC_PERIODIC = 2, BC_FIXED = 3 };

constexpr int kTile = 8;        // tile edge of the wavefront sweep
constexpr int kMaxWaves = 10;   // waves per sweep workgroup (one ray each at a time)

// Face planes (SweepArgs::face): one slot holds the vertices (a, b), a = -1 .. n_a - 1,
// b = -1 .. n_b - 1, of the two axes other than q (a: y for q = x, else x; b: z for
// q = x or y, else y), laid out so that a tile reads and writes aligned runs:
//   [0, 64 nblk)          a, b >= 0 in 8 x 8 blocks [b / 8][a / 8][b % 8][a % 8]
//   [64 nblk, 72 nblk)    every block's last column (a % 8 == 7) again, [b / 8][a / 8][b % 8]
//   then n_a + 1 values   the row b = -1 (a = -1 .. n_a - 1)
//   then n_b values       the column a = -1 (b = 0 .. n_b - 1)
// with nblk = ceil(n_a / 8) ceil(n_b / 8); a slot is padded to a multiple of 64 values.
struct FacePlane {
    int na, nb, nba, nblk;
    __host__ __device__ FacePlane(int na_, int nb_)
        : na(na_), nb(nb_), nba((na_ + 7) >> 3), nblk(((na_ + 7) >> 3) * ((nb_ + 7) >> 3)) {}
    __host__ __device__ int64_t slot() const { return ((int64_t)nblk * 72 + na + 1 + nb + 63) / 64 * 64; }
    // vertex (a, b), a, b >= -1
    __host__ __device__ int at(int a, int b) const
    {
        if (b < 0) return nblk * 72 + a + 1;
        if (a < 0) return nblk * 72 + na + 1 + b;
        return (((b >> 3) * nba + (a >> 3)) << 6) + ((b & 7) << 3) + (a & 7);
    }
    // the copy of vertex (a, b) with a % 8 == 7, a, b >= 0, among the blocks' last columns
    __host__ __device__ int col(int a, int b) const { return (nblk << 6) + (((b >> 3) * nba + (a >> 3)) << 3) + (b & 7); }
    // first value of the block of tile (ta, tb) (vertex (8 ta + u, 8 tb + w) is at + 8 w + u),
    // and of its last column's copy (vertex (8 ta + 7, 8 tb + w) is at + w)
    __host__ __device__ int blk(int ta, int tb) const { return (tb * nba + ta) << 6; }
    __host__ __device__ int colblk(int ta, int tb) const { return (nblk << 6) + ((tb * nba + ta) << 3); }
};

// Geometry of one ray's upwind short characteristic on a uniform grid
// (section 3.3): identical for every vertex, so computed once on the host.
struct RayGeo {
    int d, a, b;      // axis whose face plane is crossed first going upwind; the others (a < b)
    int oct;          // octant: bit q set when the direction is negative along axis q
    int gidx;         // index of the ray in the caller's (or the generated) order
    int pad;
    double s;         // path length from the upwind face point to the vertex
    double w4[4];     // bilinear weights at upwind offsets (0,0) (1,0) (0,1) (1,1) along (a, b)
    double wk;        // quadrature weight
    double mu[3];     // direction cosines
    double fa, fb;    // fractional offsets of the upwind face point along a and b
};

// Everything a sweep kernel reads about the problem; passed by value.
template <typename Real>
struct SweepArgs {
    int n[3];
    int nf, na, R;            // bins, rays, rays per octant
    int nt[3];                // tiles per axis
    int bc_lo[3], bc_hi[3];
    int periodic[3];
    int64_t cells;
    int64_t plane[3];         // vertices in the plane normal to each axis
    int64_t pplane[3];        // values per slot of the face planes (FacePlane::slot)
    const RayGeo *rays;       // [na], octant-major
    const Real *chi;          // [nf][cells]
    const double *S;          // [nf][cells] source function (always FP64)
    const double *B;          // [nf][cells]
    const double *fixed[6];   // FIXED faces (real coordinates), or null
    Real *face[3];            // [nf][na][nt_q][pplane_q]: slot t holds the plane at flipped
                              // coordinate t * tile - 1 along q (slot 0: the ghost plane); its
                              // vertices inside the grid are written by the tiles, its ghost
                              // vertices before the sweep (I in the plain form, D = I - S in
                              // the difference form)
    double *wrap[3];          // [nf][na][2][plane_q]: periodic memory (I), slot = parity
    Real *part;               // [8][nq][nfc][cells] per-octant partial sums of w I (or w D)
    int f0, nfc;              // bins f0 .. f0 + nfc - 1 are swept by this call
    const int *tiles;         // packed (tx | ty << 10 | tz << 20), sorted by tx + ty + tz
    int stage_off, stage_cnt;
    int stage;                // tx + ty + tz of the tiles of this launch
    const int *frozen;        // [nf]
    const int *parity;        // [nf]: periodic slot read this sweep
    const int *stage_tab;     // [nstages + 1] offsets of the stages in tiles (batched launches)
    int nstages;
    int order;                // 0: first-order segments, 1: second order (Bezier source)
    int noct;                 // octants swept: 8, or 4 (the rays going up, octants 0 .. 3)
};

// One step of the plane-ordered sweep (monotone quadratic upwind intensity): every
// ray advances one plane along the axis its short characteristic crosses first.
// Rays are grouped in classes c = octant * 3 + d; a class's partial sums go to their
// own slot, so every vertex of a slot is written once per sweep.
constexpr int kPlaneTile = 16;     // in-plane tile edge of a plane-step workgroup
constexpr int kPlaneParts = 24;    // partial-sum slots: 8 octants x 3 first-crossed axes

template <typename Real>
struct PlaneArgs {
    int n[3];
    int nf, na;
    int periodic[3];
    int bc_lo[3], bc_hi[3];
    int64_t cells;
    const RayGeo *rays;       // [na]
    const int *cls_off;       // [25]: class c holds cls_rays[cls_off[c] .. cls_off[c + 1])
    const int *cls_rays;      // [na], ascending within a class
    const Real *chi;          // [nf][cells]
    const double *S;          // [nf][cells]
    const double *B;          // [nf][cells]
    const double *fixed[6];   // FIXED faces (real coordinates), or null
    Real *planes;             // [nf][na][2][pmax]: two planes per ray (I, or D = I - S in the
                              // difference form), indexed by the flipped in-plane coordinates
                              // (a fastest); plane t is written to slot (t + parity n_d) & 1
    int64_t pmax;
    double *wrapI;            // [nf][na][pmax] difference form: I on each ray's last plane
                              // (the next sweep's ghost plane on a periodic d axis), or null
    Real *part;               // [24][nfc][cells]
    int f0, nfc;
    const int *frozen;        // [nf]
    const int *parity;        // [nf]: sweeps run so far, modulo 2
    int tiles_a[3];           // per first-crossed axis d: in-plane tiles along a
    int ntiles[3];            // per d: in-plane tiles
};

// Gauss-Seidel ALI (rt_gs.hip): the rays going up are swept over the whole grid with
// the tile kernel (octants 0 .. 3); the rays going down then advance from the top
// plane down.  Launch t recomputes plane nz - t with its updated S and computes plane
// nz - 1 - t with the current S; the update of that plane follows.  Rays that cross a
// z face first ("steep") take 16 x 16 tiles of the plane; the others ("shallow",
// first-crossed axis d = x or y) depend on vertices of their own plane and run as a
// chain along d in one workgroup, lanes along the other in-plane axis e.
constexpr int kGsTile = 16;       // in-plane tile edge of a steep-ray workgroup
constexpr int kGsMaxLanes = 256;  // largest extent along e of a chain (4 vertices per lane)
constexpr int kGsMaxDown = 256;   // largest number of rays going down

template <typename Real>
struct GsArgs {
    int n[3];
    int nf, na;
    int periodic[3];
    int bc_lo[3], bc_hi[3];
    int64_t cells, pxy;           // vertices of the grid and of one z plane
    const RayGeo *rays;           // [na]
    const int *down;              // [nd] rays going down: the shallow ones first
    int nd, ns;                   // rays going down, shallow ones among them
    const Real *chi;              // [nf][cells]
    double *S;                    // [nf][cells] source function, updated plane by plane
    const Real *chi_t;            // [nf][nz][nx][ny] chi with y fastest (chains along x)
    double *S_t;                  // [nf][nz][nx][ny] S with y fastest, kept with S
    const double *B, *eps, *lam;  // [nf][cells]
    const double *fixed[6];       // FIXED faces (real coordinates), or null
    double *wrap[3];              // periodic memory, the layout of SweepArgs::wrap
    Real *planes;                 // [nf][nd][2][pxy] final values (I, or D = I - S) of each
                                  // downward ray on plane k in slot k & 1; steep rays in
                                  // real layout (x fastest), shallow rays along e fastest
    Real *part;                   // [nd][nf][pxy] w I (w D) of the plane being computed
    Real *coef;                   // [nf][ns][pxy][4] chain coefficients E_n, Q_n, E_o, Q_o
    Real *gh;                     // [nf][ns][4][nmax] chain ghosts: boundary-lane neighbours
                                  // on kn and ko per column, the column before the first
    void *ghS;                    // double [nf][ns][2][nmax]: S on the chain's outgoing face
                                  // along e (per column) and on its last column (per pe)
    int nmax;                     // max(nx, ny)
    int steep_blocks;             // workgroups of the steep tiles in a launch (a multiple of 8)
    const Real *part_up;          // [8][nf][cells] per-octant partials of the upward sweep
    double *J;                    // [nf][cells] the J each vertex was updated with
    const int *frozen;            // [nf]
    const int *parity;            // [nf] periodic slot read this iteration
    unsigned long long *blockmax; // [nf][nblk] residual maxima (bit patterns), zeroed per iteration
    int nblk;
    int tiles_x, ntiles;          // steep-ray tiles along x and per plane
};

// Dependency state of the persistent sweep: one completion flag per (bin, octant,
// tile) holding the epoch of the sweep that last finished it, one ticket counter per
// octant and the epoch itself, both in device memory: a small kernel before each
// sweep zeroes the counters and advances the epoch, so a sweep replayed from a
// captured graph gets a new epoch and fresh counters like one launched directly.
struct DagArgs {
    int *counter;             // [8] tickets per octant, [8] the epoch of the current sweep
    int *done;                // [nf][8][ntiles]
    int *err;                 // set when a dependency wait ran out
    uint64_t wait_ticks;      // bound of one wait in wall-clock ticks
    int ntiles;
    int nt0, nt1;             // tiles along x and y
    __host__ __device__ int tile_id(int tx, int ty, int tz) const { return (tz * nt1 + ty) * nt0 + tx; }
};

// Device-side control block of the Lambda iteration.
struct AliCtl {
    int *frozen;              // [nf]
    int *parity;              // [nf]
    int *iters;               // [nf]
    double *resid;            // [nf]
    unsigned long long *blockmax;  // [nf][nblk] per-block max of |dS|/S as bit patterns
    int nblk;                 // update blocks per bin
    int *flags;               // [0] all bins stopped, [1] non-finite residual
};

constexpr int kUpdateBlocks = 1024;  // update-kernel blocks per bin (grid-stride)
constexpr int kBatchUpdateBlocks = 128;  // per bin and problem in a batched update

// One problem of a batched Jacobi update (rt_ali_solve_batch).
struct BatchUpdate {
    const void *part;         // Real [8][nf][cells]
    const double *B, *eps, *lam;
    double *S64, *J;
    int64_t cells;
    int nf, dform;
    AliCtl ctl;               // ctl.nblk = kBatchUpdateBlocks
    double delta_c;           // stopping rule of this problem's solve
    int per_bin_stop, fixed_mode;
};

// Kernel launchers (rt_kernels.hip).  All return hipError_t of the launch.
// nq = 1: partial sums of w I (or w D); nq = 10: also w mu I and w mu mu I (moments)
hipError_t launch_sweep_stage_f64(const SweepArgs<double> &A, int waves, int nq, hipStream_t st);
hipError_t launch_sweep_stage_f32(const SweepArgs<float> &A, int waves, int nq, hipStream_t st);
// dynamic LDS bytes of one sweep workgroup with the given number of waves
size_t sweep_lds_bytes(int real_bytes, int waves, int nq, bool multi, int order);
hipError_t launch_dag_begin(int *counter, hipStream_t st);
hipError_t launch_sweep_persistent_f64(const SweepArgs<double> &A, const DagArgs &D, int waves, int blocks_per_octant,
                                       hipStream_t st);
hipError_t launch_sweep_persistent_f32(const SweepArgs<float> &A, const DagArgs &D, int waves, int blocks_per_octant,
                                       hipStream_t st);
hipError_t persistent_blocks_per_cu(int real_bytes, int waves, int *blocks);

// Batched persistent sweep (rt_ali_solve_batch over problems with the persistent
// schedule).  An item is a tile of one bin of one member: the member's index in the
// class, the bin, and the tile's position in the member's tile list.  Items are listed
// by stage (tx + ty + tz), then member, bin and tile.
struct PersistItem {
    int member, f, tile, pad;
};
// A member's dependency state: its completion flags [nf][8][ntiles] and its counter
// array, whose [8] is the member's epoch (advanced before every sweep).
struct PersistMember {
    int *done;
    int *counter;
    int ntiles, nt0, nt1, pad;
};
// dag_begin for the batch (class tickets zeroed, every member's epoch advanced), then
// one persistent launch of 8 x bpo workgroups over nitems items.
hipError_t launch_sweep_persistent_batch_f64(const SweepArgs<double> *args, const PersistMember *mem,
                                             const PersistItem *items, int nitems, int nmem, int *counter, int *err,
                                             uint64_t wait_ticks, int waves, int bpo, hipStream_t st);
hipError_t launch_sweep_persistent_batch_f32(const SweepArgs<float> *args, const PersistMember *mem,
                                             const PersistItem *items, int nitems, int nmem, int *counter, int *err,
                                             uint64_t wait_ticks, int waves, int bpo, hipStream_t st);
hipError_t persistent_batch_blocks_per_cu(int real_bytes, int waves, int *blocks);

hipError_t launch_lambda_star(const int n[3], const int bc_lo[3], const int bc_hi[3], int nf, int na, int order,
                              const RayGeo *rays, const double *chi, double *lam, hipStream_t st);

// Cold periodic memory: every periodic slot about to be read holds S of the wrapped vertex.
template <typename Real>
hipError_t launch_periodic_cold(const SweepArgs<Real> &A, hipStream_t st);

// Ghost vertices of the padded face planes of the bins f0 .. f0 + nfc - 1, for the
// sweep about to run.
template <typename Real>
hipError_t launch_ghost_fill(const SweepArgs<Real> &A, hipStream_t st);

// Batched launches over the problems of one batch class (device arrays of per-problem
// arguments; sizes are the maxima over the problems).
hipError_t launch_sweep_batch_stage_f64(const SweepArgs<double> *args, int nprob, int s, int max_items, int waves,
                                        bool multi, int order, hipStream_t st);
hipError_t launch_sweep_batch_stage_f32(const SweepArgs<float> *args, int nprob, int s, int max_items, int waves,
                                        bool multi, int order, hipStream_t st);
template <typename Real>
hipError_t launch_ghost_fill_batch(const SweepArgs<Real> *args, int nprob, int64_t max_entries, int max_na,
                                   hipStream_t st);
template <typename Real>
hipError_t launch_ali_update_batch(const BatchUpdate *bu, int nprob, int nblk, int max_nf, hipStream_t st);
hipError_t launch_ali_finalize_batch(const BatchUpdate *bu, int nprob, int *done, hipStream_t st);

// npart: partial-sum slots summed per vertex (8 octants, or kPlaneParts)
template <typename Real>
hipError_t launch_partial_sum(const Real *part, int npart, const double *S, int dform, int nf, int64_t cells,
                              const int *frozen, double *J, hipStream_t st);

template <typename Real>
hipError_t launch_ali_update(const Real *part, int npart, int dform, int nf, int64_t cells, const double *B,
                             const double *eps, const double *lam, double *S64, double *J,
                             AliCtl ctl, hipStream_t st);

// Plane-ordered sweep (rt_plane.hip): one step t of every active bin's rays, and the
// cold periodic memory (the slot read at t = 0 holds S of the wrapped vertex).
// nq = 1: the class partials of w I (or w D); nq = 10: also w mu_i I and w mu_i mu_j I,
// slots [class][q]
template <typename Real>
hipError_t launch_plane_step(const PlaneArgs<Real> &A, int t, int nq, hipStream_t st);
template <typename Real>
hipError_t launch_plane_cold(const PlaneArgs<Real> &A, hipStream_t st);

// Gauss-Seidel backward sweep (rt_gs.hip): launch t of the plane pass, the update of
// plane k, and the cleared residual maxima of an iteration.  before/after (or null):
// events that take the start and end time of the chain launch of step t.
template <typename Real>
hipError_t launch_gs_plane(const GsArgs<Real> &A, int t, hipStream_t st, hipEvent_t before = nullptr,
                           hipEvent_t after = nullptr);
template <typename Real>
hipError_t launch_gs_update(const GsArgs<Real> &A, int k, hipStream_t st);
hipError_t launch_gs_clear(unsigned long long *blockmax, int64_t n, hipStream_t st);
// [nf][nz][ny][nx] -> [nf][nz][nx][ny]
template <typename T>
hipError_t launch_gs_transpose(const T *src, T *dst, int nf, const int n[3], hipStream_t st);

hipError_t launch_ali_finalize(AliCtl ctl, int nf, double delta_c, int per_bin_stop, int fixed_mode,
                               hipStream_t st);
hipError_t launch_flip_parity(int *parity, const int *frozen, int f0, int cnt, hipStream_t st);

// Angle-set sums added to the moments of the difference form: m[0] = 1 (J = S + sum w D),
// m[1..3] = sum w mu_i, m[4..9] = sum w mu_i mu_j (xx yy zz xy xz yz).
struct MomConst {
    double m[10];
};
// npart: partial-sum slots per quantity (8 octants, or kPlaneParts classes)
template <typename Real>
hipError_t launch_moments_combine(const Real *part, int npart, const double *S, int dform, int f0, int nfc, int nf,
                                  int64_t cells, const MomConst &mc, double *J, double *H, double *K, double *tmp,
                                  hipStream_t st);
hipError_t launch_moments_q(const double *tmp, int f0, int nfc, const int n[3], const double h[3], const int per[3],
                            const double *chi, const double *eps, const double *B, double *Qt, hipStream_t st);
hipError_t launch_moments_integrate(const double *tmp, const double *Qt, const double *w_nu, int f0, int nfc,
                                    int64_t cells, int first, double *J_int, double *H_int, double *K_int,
                                    double *Q_int, hipStream_t st);
hipError_t launch_eddington(const double *J_int, const double *K_int, int64_t cells, double *f_int, hipStream_t st);
hipError_t launch_sum(const double *x, int64_t n, double scale, double *partial, int nblk, double *out, hipStream_t st);
hipError_t launch_convert_f32(const double *src, float *dst, int64_t n, hipStream_t st);
hipError_t launch_convert_f64(const float *src, double *dst, int64_t n, hipStream_t st);
hipError_t launch_warm_start(const double *B, const double *eps, const double *J, double *S, int64_t n,
                             hipStream_t st);

}  // namespace rtsc
