// Internal definitions shared by the HIP translation units of libp3msr.
//
// Data layout in HBM (all built per call from the caller's arrays):
//   sp[p]        double4 (x, y, z, w) of the p-th particle in tile -> subtile
//                order, positions wrapped into [0, box); w = mu (FP64 path) or
//                the bits of float mu in the low word (FP32 path)
//   perm[p]      original index of sorted particle p
//   sel[p]       receiver selector of sorted particle p (active flag or rung)
//   cell_start[c] first sorted index of fine cell c (c = tile*ns^3 + subtile),
//                cell_start[ncells] = n
//   act_pos[]    sorted indices of the receivers, subset-major, tile order
//   clusters[]   receiver groups of <= csize (8..64) particles inside one tile
//   items[]      (cluster, neighbour-tile range, subtile range) work units,
//                the items of one cluster consecutive
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include <cstddef>
#include <cstdint>

namespace p3m {

constexpr int kWave = 64;
constexpr int kScanBlock = 256;             // threads per scan block
constexpr int kScanPerThread = 16;          // elements per scan thread
constexpr int kScanTile = kScanBlock * kScanPerThread;
constexpr int kForceBlock = 256;            // 4 waves, each with its own work item
constexpr int kSupplierPad = 128;           // zeroed records after the sorted particles
constexpr int kFineSide = 8;                // fine order: 8x8x8 sub-cells per subtile
constexpr int kFineBins = kFineSide * kFineSide * kFineSide;
constexpr int kFineMin = 8;                 // subtiles with at most this many keep their order
constexpr int kFineBig = 1024;              // larger subtiles are ordered by a whole block
constexpr int kFineWaves = 4;               // tiles (one per wave) per fine-order block
constexpr int kFinishWaves = 4;             // waves per block of the cluster box kernel
constexpr int kFinishLanes = 8;             // lanes per cluster in the box kernel
constexpr int kListCap = 224;               // screened supplier records per wave (LDS)
constexpr int kListCapF32 = 176;            // the same for the six-wave FP32 forward kernel
constexpr int kListCapAdjoint = 128;        // the same for the adjoint (entries carry weights)
constexpr int kListSlack = 32;              // records past the cap for look-ahead reads (3*8 used)

// Geometry of one call.  Tiles are cubes of side box/nt >= r_cut; each tile
// holds ns^3 subtiles; fine cells are the subtiles, nc = nt*ns per dimension.
struct Geom {
    double box, inv_box;
    double rc2;        // r_cut^2: the pair test is r^2 < rc2 (strict)
    double tile;       // tile side
    double sub;        // subtile side
    double inv_cell;   // nc / box
    double cull2;      // (r_cut + margin)^2 for conservative subtile culling
    double k1;         // 1 / (2 x_s)
    double k2;         // -log2(e) / (4 x_s^2): exp(-u^2) = 2^(r^2 k2)
    double kb;         // 1 / (2 sqrt(pi) x_s^3), Gaussian term of the pair Jacobian
    double x_s;
    int nt, ns, nc, ns3, nt3;
    float k1f, kbf;    // FP32 copies of k1 and kb
    float c2f;         // 1 / (4 x_s^2): t = u^2 = r^2 c2
    float c3f;         // 1 / (8 x_s^3): g(u) / r^3 = r^-3 + H(t) c3
    double c2, c3;     // FP64 copies of c2f and c3f
    double h64[18];    // FP64 H coefficients (kernel argument, so they sit in SGPRs)
    double eps_b;      // B-spline softening length (0: point particles)
    double eps_b2;     // eps_b^2: pairs with r^2 < eps_b2 take the softened form
    double inv_eps_b;  // 1 / eps_b
    double ks3, ks5;   // 32 / eps_b^3, 32 / eps_b^5
    float inv_eps_bf;  // FP32 copy of inv_eps_b
};

struct Cluster {
    int tile;     // tile index (tx*nt + ty)*nt + tz
    int subset;   // receiver subset (batched calls)
    int begin;    // first entry in act_pos / rp / rperm
    int count;    // 1..csize receivers
    double lo[3]; // bounding box of the receivers (wrapped positions)
    double hi[3];
};

// Work item: receivers of one cluster against suppliers in neighbour tiles
// [t0, t1) of the 27-tile stencil (t = (ox+1)*9 + (oy+1)*3 + (oz+1)) and,
// when t1 == t0 + 1, only subtiles [s0, s1) of that tile.
struct Item {
    int cluster;
    int tiles;    // t0 | t1 << 8
    int subs;     // s0 | s1 << 16
    int sole;     // kItemSole: the only item of its cluster (its sums are stored, not
                  // added); kItemFirst: the cluster's first item
};
constexpr int kItemSole = 1;
constexpr int kItemFirst = 2;

struct Counters {
    unsigned long long interactions;
    unsigned long long candidates;
    unsigned long long steps;        // wave steps over suppliers
    unsigned long long screened;     // supplier records tested against cluster boxes
    unsigned long long rare;         // mutual kernel: wave steps that took the FP64 path
    unsigned long long scan_stall;   // single-pass scans whose look-back hit its poll limit
    unsigned long long pad[2];
};
static_assert(256 % sizeof(Counters) == 0, "Counters copies are 256 B apart");

// The pair kernels add their waves' counts into one Counters copy per XCD,
// each in a 256 B line of its own (the readers sum the copies): one copy for
// every wave would queue their atomics on one cache line at the end of the
// launch.
constexpr int kCounterCopies = 8;
constexpr int kCounterStride = 256 / sizeof(Counters);

enum SelKind { SEL_ALL = 0, SEL_MASK = 1, SEL_RUNG = 2 };

// ---- work items ---------------------------------------------------------------

__device__ inline int neighbour_tile(int tile, int t, const Geom &g) {
    int tx = tile / (g.nt * g.nt), ty = (tile / g.nt) % g.nt, tz = tile % g.nt;
    int nx = tx + t / 9 - 1, ny = ty + (t / 3) % 3 - 1, nz = tz + t % 3 - 1;
    nx += nx < 0 ? g.nt : (nx >= g.nt ? -g.nt : 0);
    ny += ny < 0 ? g.nt : (ny >= g.nt ? -g.nt : 0);
    nz += nz < 0 ? g.nt : (nz >= g.nt ? -g.nt : 0);
    return (nx * g.nt + ny) * g.nt + nz;
}

// Greedy grouping of the 27 neighbour tiles into items of about `target`
// supplier candidates (before subtile culling); a tile holding more than
// `target` particles is split by subtile ranges.  Returns the item count and
// writes the items when `out` is non-null.  At most 2 per stencil tile plus
// one with one subtile per tile (a flush and the tile itself), at most
// 1 + ns^3 per tile plus one otherwise (plan_items_bound).
//
// half != 0 (pairs evaluated once, for both partners): only the upper half
// of the stencil, t = 13 .. 26, whose periodic mirror images are the lower
// half; in the own tile (t = 13) only the particles after the cluster count,
// and every cluster gets at least one item, so that its own pairs are
// evaluated.  The first item of a cluster carries kItemFirst.
// Upper bound on the items plan_items gives one cluster.
inline long long plan_items_bound(int ns3, int half) {
    const long long tiles = half ? 14 : 27;
    return tiles * (ns3 == 1 ? 2 : 1 + ns3) + 2;
}

__device__ inline int plan_items(int cidx, const Cluster &cl, const int *__restrict__ cs,
                                 const Geom &g, int target, Item *out, int sole, int half) {
    int n = 0, acc = 0;
    const int t_begin = half ? 13 : 0;
    int t0 = t_begin;
    auto emit = [&](int a, int b, int s0, int s1) {
        if (out) {
            Item it;
            it.cluster = cidx;
            it.tiles = a | (b << 8);
            it.subs = s0 | (s1 << 16);
            it.sole = sole | (n == 0 ? kItemFirst : 0);
            out[n] = it;
        }
        ++n;
    };
    for (int t = t_begin; t < 27; ++t) {
        int nb = neighbour_tile(cl.tile, t, g);
        int w = cs[(size_t)(nb + 1) * g.ns3] - cs[(size_t)nb * g.ns3];
        if (half && t == 13) w = cs[(size_t)(nb + 1) * g.ns3] - (cl.begin + cl.count);
        if (w > target) {
            if (acc > 0) emit(t0, t, 0, g.ns3);
            int parts = min((w + target - 1) / target, g.ns3);
            for (int q = 0; q < parts; ++q)
                emit(t, t + 1, q * g.ns3 / parts, (q + 1) * g.ns3 / parts);
            t0 = t + 1;
            acc = 0;
        } else if (acc + w > target) {
            emit(t0, t, 0, g.ns3);
            t0 = t;
            acc = w;
        } else {
            if (acc == 0 && w == 0) t0 = t + 1;   // skip leading empty tiles
            acc += w;
        }
    }
    if (acc > 0) emit(t0, 27, 0, g.ns3);
    if (half && n == 0) emit(13, 14, 0, g.ns3);
    return n;
}

// ---- launchers (host functions defined in the .hip files) -----------------

// sort.hip
hipError_t launch_fill_i32(int *p, int v, size_t n, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s);
// cell key and rank inside the cell of every particle (cell_count zeroed)
hipError_t launch_keys(const double *pos, int n, const Geom &g, int *key, int *rank,
                       int *cell_count, hipStream_t s);
size_t scan_block_sums_needed(size_t n);
// exclusive scan of n int32 values; out has n+1 entries (out[n] = total).
// in may equal out.
hipError_t launch_scan(const int *in, int *out, size_t n, int *block_sums, hipStream_t s);
// the same in one launch (decoupled look-back) for up to 64 tiles of
// kScanTile values, else as launch_scan (with bsum): status holds
// scan1_status_needed(n) entries and *ctr one int, both zeroed before the
// launch; a look-back that waited past its poll limit raises *stall
size_t scan1_status_needed(size_t n);
hipError_t launch_scan1(const int *in, int *out, size_t n, unsigned long long *status, int *ctr,
                        unsigned long long *stall, int *bsum, hipStream_t s);
// scatter into tile -> subtile order: particles of subtiles that the fine
// order leaves as they are (at most max(csize, kFineMin)) go to sp2/perm2/sel2,
// the others to sp/perm/sel_s for launch_fine_order
// stable: ranks from launch_stable_ranks (already in fine order), so every
// subtile goes to sp2/perm2/sel2 and no fine-order pass follows
hipError_t launch_scatter(const double *pos, const double *mass, const uint8_t *sel, int n,
                          const Geom &g, const int *key, const int *rank,
                          const int *cell_start, int fp32, int csize, bool stable, double4 *sp,
                          int *perm, uint8_t *sel_s, double4 *sp2, int *perm2, uint8_t *sel2,
                          hipStream_t s);
// Deterministic mode: rank[i] = place of particle i in its cell when the
// cell's particles are ordered by (fine sub-cell, index) (cell_start: the
// scanned cell counts; key: launch_keys' cell keys).  Scratch: k64a/k64b n
// each, va/vb n each, hist stable_rank_hist_ints(n) + 1, bsum for a scan of
// that many values.
size_t stable_rank_hist_ints(int n);
hipError_t launch_stable_ranks(const double *pos, int n, const Geom &g, const int *key,
                               const int *cell_start, unsigned long long *k64a,
                               unsigned long long *k64b, int *va, int *vb, int *hist, int *bsum,
                               int *rank, hipStream_t s);
// Deterministic mode: the sums of clusters with several items from the
// items' partial slots (partials[(item * csize + receiver) * 3 + c]), added
// in item order into out (item_off: the scanned item counts per cluster)
hipError_t launch_item_reduce(const Cluster *clusters, const int *n_clusters_dev, int bound,
                              const int *item_off, const double *partials, int csize,
                              const int *rperm, double *out, long long out_stride,
                              hipStream_t s);
// reorder the particles of every subtile by the Morton index of their fine
// sub-cell (sp/perm/sel -> sp2/perm2/sel2; sel == nullptr: no selector;
// fkey/frank: n ints of scratch).  launch_big_list lists the subtiles above
// kFineBig particles in big_list (1 + n / kFineBig ints, big_list[0] zeroed
// before it); launch_fine_order_medium orders the others, and
// launch_fine_order_big the listed ones (after launch_big_list; the two
// orderings touch different subtiles and may run at the same time)
hipError_t launch_big_list(const int *cell_start, const Geom &g, int *big_list, hipStream_t s);
hipError_t launch_fine_order_medium(const double4 *sp, const int *perm, const uint8_t *sel,
                                    const int *cell_start, const Geom &g, int *fkey, int *frank,
                                    double4 *sp2, int *perm2, uint8_t *sel2, int csize,
                                    hipStream_t s);
hipError_t launch_fine_order_big(const double4 *sp, const int *perm, const uint8_t *sel,
                                 const int *cell_start, const Geom &g, int *fkey, int *frank,
                                 double4 *sp2, int *perm2, uint8_t *sel2, int n,
                                 const int *big_list, hipStream_t s);
hipError_t launch_flags(const uint8_t *sel_s, int n, int n_sub, int kind,
                        const uint8_t *thr_host, int *flags, hipStream_t s);
hipError_t launch_compact(const int *scan, int n, int n_sub, int *act_pos, hipStream_t s);
// *a, *b, *c -> host_out[0..2] (pinned host memory)
hipError_t launch_totals(const int *a, const int *b, const int *c, int *host_out,
                         hipStream_t s);
// scan == nullptr (one subset, every particle a receiver): receivers are the
// sorted particles themselves
hipError_t launch_cluster_count(const int *cell_start, const int *scan, int n, int n_sub,
                                const Geom &g, int csize, int *ncl, hipStream_t s);
hipError_t launch_cluster_write(const int *cell_start, const int *scan, const int *cl_off,
                                int n, int n_sub, const Geom &g, int csize, Cluster *clusters,
                                hipStream_t s);
// half != 0: items over the upper half of the neighbour stencil only, for
// the pair kernel that evaluates each pair once for both partners
hipError_t launch_item_count(const Cluster *clusters, const int *n_clusters_dev,
                             int cluster_bound, const int *cell_start, const Geom &g,
                             int target, int half, int *item_cnt, hipStream_t s);
// every cluster's items at their offsets item_off (the scanned counts; the
// array holds them all); the cluster count is read on the device.  host_tot
// (nullable, pinned): receives the receiver total *tot_recv, the cluster
// count and the item total *tot_items.
hipError_t launch_item_write(const Cluster *clusters, const int *n_clusters_dev, int bound,
                             const int *cell_start, const Geom &g, int target, int half,
                             const int *item_off, Item *items, const int *tot_recv,
                             const int *tot_items, int *host_tot, hipStream_t s);
// 32-bin histogram of particles per tile (log2 bins; bin 0: empty tiles),
// the occupancy signature the autotuner files its results under
hipError_t launch_tile_hist(const int *cell_start, const Geom &g, int *hist32, hipStream_t s);
hipError_t launch_gather_weights(const double *grad_acc, const uint8_t *sel_s, const int *perm,
                                 int n, int fp32, double4 *wa, hipStream_t s);
// per cluster: receivers copied to rp / rperm / rwa (indexed like act_pos;
// rp == nullptr: no copy, act_pos == nullptr as scan == nullptr above) and the
// bounding box filled in; *n_clusters_dev clusters, at most `bound`
hipError_t launch_cluster_finish(Cluster *clusters, const int *n_clusters_dev, size_t bound,
                                 int csize, const int *act_pos, const double4 *sp,
                                 const int *perm, const double4 *wa, double4 *rp, int *rperm,
                                 double4 *rwa, hipStream_t s);
// up to kFillMax int regions set to their values in one launch
constexpr int kFillMax = 8;
struct FillSet {
    int *p[kFillMax];
    size_t n[kFillMax];
    int v[kFillMax];
    int count;
    void add(int *ptr, size_t len, int val) {
        p[count] = ptr;
        n[count] = len;
        v[count] = val;
        ++count;
    }
};
hipError_t launch_fill_multi(const FillSet &f, hipStream_t s);

// force.hip
enum PairMode { FWD_F32 = 0, FWD_F64 = 1, BWD_F32 = 2, BWD_F64 = 3 };
constexpr int kXcds = 8;   // MI355X: workgroups are dealt round-robin to 8 XCDs
static_assert(kCounterCopies == kXcds, "one Counters copy per XCD");
// ints between the XCD work counters: each in a 256 B line of its own, so
// claims from different XCDs do not queue on one cache line
constexpr int kQueueStride = 64;

struct PairArgs {
    const double4 *sp;       // suppliers in sorted order
    const double4 *rp;       // receivers, indexed like act_pos
    const double4 *rwa;      // backward: receivers' w * [active] (FP32 path: float4 bits)
    const int *cell_start;
    const Cluster *clusters;
    const Item *items;
    const double4 *wa;       // backward: suppliers' w * [active], sorted (FP32: float4 bits)
    int *queue;              // kXcds work counters kQueueStride ints apart, zero at launch
    const int *rperm;        // original index of each receiver row (indexed like act_pos)
    double *out;             // n_sub x n x 3, zeroed before the launch
    long long out_stride;    // elements per subset in out (3 n)
    Counters *counters;      // kCounterCopies copies, kCounterStride apart
    // the item count, read on the device (the host need not wait for it)
    const int *n_items_dev;
    int unit_mass;           // no mass array: every mu_j is 1 (forward kernels specialise)
    int csize;               // cluster size (receivers per cluster, 8..64)
    // tabulated FP32 forward shape (kernel kind 1 or 2, see force.hip)
    const float *htab;       // NGP: tab_n values; linear: tab_n (value, slope) pairs
    float tab_scale;         // table entries per unit of r^2: tab_n / r_cut^2
    int tab_n;
    // mutual kernel: FP32 r^2 in [rc2_lo, rc2_hi) is tested again in FP64
    float rc2_lo, rc2_hi;
    // deterministic mode: items of clusters with several items store their
    // sums in partial slots ((item * csize + receiver) * 3) instead of
    // adding them with atomics (nullptr: atomics)
    double *partials;
    Geom g;
};

constexpr int kTabFloats = 4096;   // LDS floats a table may take (16 KB)
enum ShapeKind { SHAPE_POLY = 0, SHAPE_TAB_NGP = 1, SHAPE_TAB_LINEAR = 2 };
// Fills the table of H(t) (g(u) / r^3 = r^-3 + H(t) / (2 x_s)^3, t = u^2) on
// r^2 in [0, rc2): NGP holds H at the n bin centres, linear the value at the
// n + 1 nodes as (value, next - value) pairs.
hipError_t launch_build_htab(int kind, int n, const Geom &g, float *tab, hipStream_t s);
// screen != 0: every supplier is tested against the cluster's box first and
// the survivors (with the adjoint's weights) stream from LDS
// tab: ShapeKind of the FP32 forward shape (the other modes ignore it)
hipError_t launch_pairs(int mode, int screen, int tab, const PairArgs &a, int grid,
                        hipStream_t s);

// Long-range PM (pm.hip).  real: n^3 FP64 (rho, then phi), x fastest;
// spec: n^2 rows of n/2 + 1 complex FP64 (kx fastest) at a stride rounded up
// to 8; tw: n/2 twiddles; w1, k2:
// per-axis kernel tables of n values; scale = 4 pi / h^4 / n^3.
struct PmArgs {
    int n;
    double *real;
    double2 *spec;
    const double2 *tw;
    const double *w1, *k2;
    double scale;
};
hipError_t launch_pm_tables(int n, double box, double x_s, double2 *tw, double *w1, double *k2,
                            hipStream_t s);
// sort: key/rank n_part ints, count n^3 + 1 ints (scanned in place into the
// first sorted index of each node), bsum scan block sums;
// rec (CIC fractions, mu), nkey, perm, recv n_part entries in node order
hipError_t launch_pm_sort(const double *pos, const double *mass, const uint8_t *active,
                          int n_part, int n, double box, double h, int *key, int *rank,
                          int *count, int *bsum, double4 *rec, int *nkey, int *perm,
                          uint8_t *recv, hipStream_t s);
// rho (n^3, fully written) from the node-sorted records; start: the node
// starts of the sort (n^3 + 1 entries)
hipError_t launch_pm_deposit(const double4 *rec, const int *nkey, const int *start, int n_part,
                             double *rho, int n, hipStream_t s);
// ev (optional): 4 events recorded after the x, y and z passes and the y
// inverse pass
hipError_t launch_pm_fft_chain(const PmArgs &a, hipStream_t s, hipEvent_t *ev);
hipError_t launch_pm_readout(const double4 *rec, const int *nkey, const int *perm,
                             const uint8_t *recv, int n_part, const double *phi, int n,
                             double *acc, hipStream_t s);
// pair-kernel workgroups resident per CU for the variant launch_pairs would run
int pairs_blocks_per_cu(int mode, int screen, int tab, int csize, int unit_mass, int soft);
// All-active FP32 forward (bwd: the FP32 adjoint, every particle a receiver,
// weights in a.wa; f64: the FP64 kinds, the adjoint without softening) with each pair
// evaluated once for both partners (clusters
// of csize = 16, 32 or 64 receivers, items over the upper half of the
// stencil).  a.out: three FP64 arrays of a.out_stride = n sums in sorted
// order, zeroed before the launch; launch_mutual_out then writes acc_out.
hipError_t launch_pairs_mutual(const PairArgs &a, bool bwd, bool f64, int grid, hipStream_t s);
int mutual_blocks_per_cu(int csize, int unit_mass, bool bwd, bool soft, bool f64);
hipError_t launch_mutual_out(const double *sums, const int *perm, int n, double *out,
                             hipStream_t s);

// KDK step (kdk.hip).  Times in units of tau / 2, tau = dt / 2^L.
struct KdkArgs {
    double dt;
    double two_eta_eps;   // 2 eta eps of eq. rung
    double half_tau;
    int L;                // highest rung of the period
    int period;           // n_steps 2^(L+1)
    int max_rung;
    int fixed;            // 1: rungs are inputs and never change
};
hipError_t launch_kdk_assign(const double *acc, int n, const KdkArgs &k, uint8_t *rung,
                             int *max_rung, hipStream_t s);
hipError_t launch_kdk_first(double *vel, const double *acc, int n, const KdkArgs &k,
                            const uint8_t *rung, int *t_q, int *t_next, hipStream_t s);
hipError_t launch_kdk_drift(double *pos, const double *vel, int n, double tau, double box,
                            hipStream_t s);
hipError_t launch_kdk_due(const int *t_next, int n, int t, uint8_t *due, int *n_due,
                          hipStream_t s);
hipError_t launch_kdk_kick(double *vel, const double *acc, const uint8_t *due, int n, int t,
                           const KdkArgs &k, uint8_t *rung, int *t_q, int *t_next,
                           hipStream_t s);
// vel += dk acc over n x 3 values
hipError_t launch_axpy3(double *vel, const double *acc, int n, double dk, hipStream_t s);
hipError_t launch_kdk_accum(const Counters *c, unsigned long long *total, hipStream_t s);

}  // namespace p3m
