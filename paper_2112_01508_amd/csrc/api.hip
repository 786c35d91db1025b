// C ABI of libp3msr: argument checks, workspace, the launch pipeline, the
// measure-and-keep autotuner and per-call counters.
//
// Pipeline of one force call (all on the caller's stream):
//   keys      tile/subtile key per particle + rank inside its cell (atomics)
//   scan      exclusive scan of the cell histogram -> cell_start
//   scatter   particles into tile -> subtile order (section 2.1.3, memory
//             reorder of "Other optimisations")
//   flags     receiver flags per subset, scan, compaction
//   fine      inside dense subtiles, particles reordered by fine sub-cell
//   clusters  <= csize (8..64) consecutive receivers of one tile per cluster
//   items     clusters split over their 27 neighbour tiles (work estimate)
//   [read back the cluster and item totals: the only host synchronisation]
//   pairs     one persistent launch over all items; an item's sums are stored
//             (sole item of its cluster) or added with FP64 atomics
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sys/stat.h>
#include <unistd.h>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/p3msr.h"
#include "p3msr_internal.hpp"
#include "gpoly.inc"

using namespace p3m;

namespace {

thread_local std::string g_last_error = "no error";

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define P3M_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_error(P3M_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

// Tuned layouts are filed by particle count, tiles per dimension,
// precision, call kind (forward, adjoint, rung-batched) and subset count.
// When the forward's or the adjoint's winner evaluates each pair once for
// both partners, the fastest of the other layouts is filed too (the PLAIN
// kinds), for the calls that layout cannot serve: masked, tabulated-shape,
// deterministic and softened adjoint ones.
enum TuneKind {
    TUNE_FORWARD = 0,
    TUNE_ADJOINT = 1,
    TUNE_BATCHED = 2,
    TUNE_FORWARD_PLAIN = 3,
    TUNE_ADJOINT_PLAIN = 4
};
constexpr int kTuneKinds = 5;
int plain_kind(int kind) {
    return kind == TUNE_FORWARD ? TUNE_FORWARD_PLAIN
                                : (kind == TUNE_ADJOINT ? TUNE_ADJOINT_PLAIN : -1);
}
struct TuneKey {
    int64_t n;
    int nt;
    int precision;
    int kind;
    int n_sub;
    bool operator<(const TuneKey &o) const {
        return std::tie(n, nt, precision, kind, n_sub) <
               std::tie(o.n, o.nt, o.precision, o.kind, o.n_sub);
    }
    bool operator==(const TuneKey &o) const { return !(*this < o) && !(o < *this); }
};
// Device buffers of one short-range call.  base != nullptr: every buffer is
// a slice of [base, base + size), handed out anew at each call (nothing is
// freed or allocated); else each buffer grows with hipMalloc.
struct SrWork {
    DevBuf key, rank, cells, sp, perm, sel, sp2, perm2, sel2, flags, actpos, ncl, clusters,
        itemcnt, items, bsum, counters, wa, scal, rp, rperm, rwa, fbig, msum, htab;
    // deterministic mode: radix-sort keys and values (two of each), digit
    // counts, and the items' partial sums
    DevBuf det_k, det_v, det_hist, partials;
    // single-pass scans: their tile status words and tile counters
    DevBuf scan1;
    unsigned char *base = nullptr;
    size_t size = 0, used = 0;
};

struct TuneVal {
    int ns;
    int target;
    int csize;
    int screen;
};

// One result of the autotuner as kept in the persistent cache: the device,
// the key, the occupancy signature of the particle set it was timed on (the
// 32-bin histogram of particles per tile of launch_tile_hist), the layout
// and its time.
constexpr int kSigBins = 32;
struct TuneEntry {
    std::string device;
    TuneKey key{};
    int sig[kSigBins] = {};
    TuneVal val{};
    double ms = 0.0;
};

// Distance of two signatures: the L1 distance of the normalised histograms
// (0 for the same occupancy, 2 for disjoint ones).
double sig_distance(const int *a, const int *b) {
    double ta = 0, tb = 0, d = 0;
    for (int k = 0; k < kSigBins; ++k) {
        ta += a[k];
        tb += b[k];
    }
    if (ta <= 0 || tb <= 0) return ta == tb ? 0.0 : 2.0;
    for (int k = 0; k < kSigBins; ++k) d += std::fabs(a[k] / ta - b[k] / tb);
    return d;
}
// A cached layout is reused for a particle set whose signature is this close.
constexpr double kSigMatch = 0.05;

}  // namespace

struct p3m_sr_context {
    int device = 0;
    int n_cu = 0;
    // resident pair-kernel blocks per CU, per variant: mode, screen, cluster size,
    // shape, unit mass, softening
    int blocks_per_cu[4 * 2 * 4 * 3 * 4] = {};
    int mutual_blocks_per_cu[4 * 2 * 2 * 2 * 2] = {};   // by cluster size, adjoint, unit mass, softening, FP64
    // short-range workspace: grown with hipMalloc as calls need it, or (the
    // no-alloc entry point) carved from the library's fixed device array
    SrWork work, fixed;
    Counters *last_counters = nullptr;   // counters of the most recent call
    int cfg_ns = 0, cfg_target = 0, cfg_csize = 0, cfg_screen = -1;
    int cfg_shape = SHAPE_POLY, cfg_tab_n = 0;   // FP32 forward shape (p3m_sr_set_shape)
    double eps = 0.0;   // Plummer-equivalent softening length (0: point particles)
    std::map<TuneKey, TuneVal> tuned;
    // persistent autotuner cache: file (empty: none), its entries, this
    // device's identity, and what the last autotune call did
    std::string cache_path, device_id;
    std::vector<TuneEntry> cache;
    int tune_trials = 0, tune_from_cache = 0;
    p3m_sr_stats stats{};
    hipStream_t last_stream = nullptr;
    bool timing = false;
    // fixed summation order (p3m_sr_set_deterministic)
    bool deterministic = false;
    // debug limits (p3m_sr_set_debug_limits): cap on the workspace bytes held
    // through ensure() (0: none) and the number of growths allowed before
    // one is made to fail (-1: none); alloc_bytes is what ensure() holds now
    size_t dbg_max_bytes = 0;
    int dbg_fail_after = -1;
    size_t alloc_bytes = 0;
    bool timed_last = false;
    // start, pairs start, pairs end, end, sort end, sort end on the build
    // stream (the dense subtiles' fine order)
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool sort_b = false;   // ev[5] was recorded by the timed call
    hipEvent_t tot_ev = nullptr;   // after the totals of a call reach host memory
    int *host_tot = nullptr;   // pinned: receivers, clusters, items of the current call
    // long-range PM workspace and timing
    DevBuf pm_real, pm_spec, pm_tab, pm_key, pm_rank, pm_cnt, pm_rec, pm_nkey, pm_perm, pm_recv,
        pm_bsum, p3m_lr, tune_w, tune_sig;
    // p3m_force: the long-range half runs on this stream beside the short range
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // build phase: the cluster boxes and the output clear run on this stream
    // beside the item planning (forked from and joined to the call's stream)
    hipStream_t bstream = nullptr;
    hipEvent_t bfork = nullptr, bjoin = nullptr, bsort = nullptr, bsorted = nullptr;
    // with every particle a receiver: the cluster and item planning runs on
    // this stream beside the scatter and the fine order
    hipStream_t pstream = nullptr;
    hipEvent_t pfork = nullptr, pjoin = nullptr;
    p3m_lr_stats lr_stats{};
    bool lr_timed = false;
    hipStream_t lr_stream = nullptr;
    hipEvent_t lr_ev[9] = {};   // start, sort, deposit, x, y, z, y inverse, x inverse, readout
    // KDK step workspace
    DevBuf kdk_acc, kdk_lr, kdk_tq, kdk_tnext, kdk_due, kdk_scal;
    p3m_kdk_stats kdk_stats{};
};

namespace {

int ensure(p3m_sr_context *h, DevBuf &b, size_t bytes, hipStream_t s) {
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return P3M_OK;
    // work queued on the caller's stream may still use the old buffer
    P3M_HIP(hipStreamSynchronize(s));
    if (h->last_stream && h->last_stream != s) P3M_HIP(hipStreamSynchronize(h->last_stream));
    if (b.p) {
        P3M_HIP(hipFree(b.p));
        h->alloc_bytes -= b.cap;
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    if (h->dbg_fail_after == 0)
        return set_error(P3M_ENOMEM, "device workspace of %zu bytes refused (debug limit)", bytes);
    if (h->dbg_max_bytes && h->alloc_bytes + bytes > h->dbg_max_bytes)
        return set_error(P3M_ENOMEM,
                         "device workspace of %zu bytes would pass the debug limit of %zu bytes",
                         bytes, h->dbg_max_bytes);
    if (h->dbg_max_bytes && h->alloc_bytes + want > h->dbg_max_bytes) want = bytes;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return set_error(P3M_ENOMEM, "device workspace of %zu bytes could not be allocated",
                             bytes);
        }
        want = bytes;
    }
    b.cap = want;
    h->alloc_bytes += want;
    if (h->dbg_fail_after > 0) --h->dbg_fail_after;
    return P3M_OK;
}

// ---- fixed workspace of p3m_sr_force_noalloc ---------------------------------
//
// One array per GPU the library runs on, held until the process ends.  Host
// code never uses the array's name as an address: each device's address is
// looked up once (with that device current) and kept in g_scratch_dev.
// Every no-alloc call on a GPU uses the same array, so such calls must not
// overlap on one GPU (they would race); every part of it a call reads is
// written or cleared (by fill kernels) earlier in the same call.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 18;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
int scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return set_error(P3M_EUNSUPPORTED, "device %d is beyond the %d the library tracks", device,
                         kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(P3M_EHIP, "hipGetSymbolAddress(scratch) failed: %s",
                             hipGetErrorString(e));
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return P3M_OK;
}

// A buffer of the call's workspace set: a fresh 256-byte aligned slice of
// the fixed region, or a grown allocation.
int take(p3m_sr_context *h, SrWork &w, DevBuf &b, size_t bytes, hipStream_t s) {
    if (!w.base) return ensure(h, b, bytes, s);
    if (bytes == 0) bytes = 16;
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (w.used + need > w.size)
        return set_error(P3M_EUNSUPPORTED,
                         "the call needs more than the %zu bytes of the no-alloc workspace",
                         w.size);
    b.p = w.base + w.used;
    b.cap = bytes;
    w.used += need;
    return P3M_OK;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

// Largest work-item array sized by the bound on the item count; beyond it
// the call waits for the count and sizes the array exactly.
constexpr size_t kItemBoundBytes = size_t(1) << 30;

// ---- persistent autotuner cache ----------------------------------------------
//
// A JSON file holding one object per line:
//   {"device": "...", "n": N, "nt": ..., "precision": p, "kind": k, "n_sub": s,
//    "ns": ..., "target": ..., "csize": ..., "screen": ..., "ms": ..., "sig": [32 ints]}
// in an array.  Lines that do not parse are ignored.

std::string device_identity(int device) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string id = std::string(prop.gcnArchName) + "/" + prop.name + "/" +
                     std::to_string(prop.multiProcessorCount);
    for (char &c : id)
        if (c == '"' || c == '\\' || c == ' ' || c < 32) c = '_';
    return id;
}

bool valid_layout(int csize, int screen) {
    const bool cs = csize == 8 || csize == 16 || csize == 32 || csize == 64;
    return cs && screen >= 0 && screen <= 2 && (screen != 2 || csize >= 16);
}

bool parse_entry(const std::string &line, TuneEntry &e) {
    char dev[160] = {};
    long long n = 0;
    const char *p = line.c_str();
    const char *q = std::strstr(p, "{\"device\": \"");
    if (!q) return false;
    int used = 0;
    if (std::sscanf(q,
                    "{\"device\": \"%159[^\"]\", \"n\": %lld, \"nt\": %d, \"precision\": %d, "
                    "\"kind\": %d, \"n_sub\": %d, \"ns\": %d, \"target\": %d, \"csize\": %d, "
                    "\"screen\": %d, \"ms\": %lf, \"sig\": [%n",
                    dev, &n, &e.key.nt, &e.key.precision, &e.key.kind, &e.key.n_sub, &e.val.ns,
                    &e.val.target, &e.val.csize, &e.val.screen, &e.ms, &used) < 11 ||
        used == 0)
        return false;
    q += used;
    for (int k = 0; k < kSigBins; ++k) {
        int consumed = 0;
        if (std::sscanf(q, " %d%n", &e.sig[k], &consumed) < 1) return false;
        q += consumed;
        while (*q == ',' || *q == ' ') ++q;
    }
    e.device = dev;
    e.key.n = n;
    return e.key.n >= 0 && e.key.nt >= 3 && e.key.kind >= 0 && e.key.kind < kTuneKinds &&
           e.val.ns >= 1 && e.val.ns <= 16 && valid_layout(e.val.csize, e.val.screen);
}

// Entries of a cache file (false if it cannot be opened); *lines counts
// its lines.  Lines of any length are read whole.
bool read_cache_file(const std::string &path, std::vector<TuneEntry> &out, int *lines) {
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    std::string line;
    char buf[1024];
    int nl = 0;
    for (;;) {
        line.clear();
        bool got = false;
        while (std::fgets(buf, sizeof(buf), f)) {
            got = true;
            line += buf;
            if (line.back() == '\n') break;
        }
        if (!got) break;
        ++nl;
        TuneEntry e;
        if (parse_entry(line, e)) out.push_back(e);
    }
    std::fclose(f);
    if (lines) *lines = nl;
    return true;
}

void load_cache(p3m_sr_context *h) {
    h->cache.clear();
    if (h->cache_path.empty()) return;
    if (!read_cache_file(h->cache_path, h->cache, nullptr)) return;
    // this device's entries are the layouts calls use until they are re-tuned
    for (const TuneEntry &e : h->cache)
        if (e.device == h->device_id) h->tuned[e.key] = e.val;
}

void mkdir_parents(const std::string &path) {
    for (size_t k = 1; k < path.size(); ++k)
        if (path[k] == '/') (void)mkdir(path.substr(0, k).c_str(), 0755);
}

// Write the cache (a temporary file renamed over the old one); failures to
// write are ignored: the cache is an optimisation.
void save_cache(const p3m_sr_context *h) {
    if (h->cache_path.empty()) return;
    mkdir_parents(h->cache_path);
    const std::string tmp = h->cache_path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "[\n");
    for (size_t k = 0; k < h->cache.size(); ++k) {
        const TuneEntry &e = h->cache[k];
        std::fprintf(f,
                     "{\"device\": \"%s\", \"n\": %lld, \"nt\": %d, \"precision\": %d, "
                     "\"kind\": %d, \"n_sub\": %d, \"ns\": %d, \"target\": %d, \"csize\": %d, "
                     "\"screen\": %d, \"ms\": %.6g, \"sig\": [",
                     e.device.c_str(), (long long)e.key.n, e.key.nt, e.key.precision, e.key.kind,
                     e.key.n_sub, e.val.ns, e.val.target, e.val.csize, e.val.screen, e.ms);
        for (int b = 0; b < kSigBins; ++b) std::fprintf(f, b ? ", %d" : "%d", e.sig[b]);
        std::fprintf(f, "]}%s\n", k + 1 < h->cache.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), h->cache_path.c_str()) != 0) std::remove(tmp.c_str());
}

std::string default_cache_path() {
    const char *env = std::getenv("P3MSR_TUNE_CACHE");
    if (env) return env;   // empty: no persistent cache
    const char *home = std::getenv("HOME");
    if (!home || !*home) return "";
    return std::string(home) + "/.cache/p3msr/autotune.json";
}

int check_geometry(int64_t n, double box, double x_s, double r_cut) {
    if (n < 0) return set_error(P3M_EINVAL, "n must be >= 0 (got %lld)", (long long)n);
    if (n > (int64_t)0x7fffffff - 64)
        return set_error(P3M_EUNSUPPORTED, "n = %lld exceeds the 2^31 particle limit",
                         (long long)n);
    if (!(box > 0) || !std::isfinite(box)) return set_error(P3M_EINVAL, "box must be > 0");
    if (!(x_s > 0) || !std::isfinite(x_s)) return set_error(P3M_EINVAL, "x_s must be > 0");
    if (!(r_cut > 0) || !std::isfinite(r_cut))
        return set_error(P3M_EINVAL, "r_cut must be > 0");
    if (!(r_cut < 0.5 * box))
        return set_error(P3M_EINVAL, "r_cut must be < box/2 for a single nearest image");
    if (std::floor(box / r_cut) < 3.0)
        return set_error(P3M_EINVAL, "need at least 3 tiles of side >= r_cut per dimension");
    // the kernel-shape fits cover u = r / (2 x_s) <= 2.25, the paper's r_cut = 4.5 x_s
    if (r_cut > 4.5 * x_s * (1.0 + 1e-12))
        return set_error(P3M_EUNSUPPORTED, "r_cut = %g x_s exceeds the supported 4.5 x_s",
                         r_cut / x_s);
    return P3M_OK;
}

// Tiles per dimension: as many as possible with side >= r_cut (kept a hair
// above r_cut so that rounding in the cell assignment cannot put a partner
// two tiles away), capped so that the cell index fits in 32 bits.
int tiles_per_dim(double box, double r_cut) {
    double q = std::floor(box / (r_cut * (1.0 + 1e-12)));
    int nt = (int)std::min(q, 1024.0);
    while (nt > 3 && box / nt < r_cut * (1.0 + 1e-12)) --nt;
    return nt < 3 ? 3 : nt;
}

int pick_subtiles(int nt, int64_t n, int requested) {
    int ns = requested;
    if (ns <= 0) {
        // default before tuning: finer subtiles when tiles hold more particles
        double per_tile = (double)n / ((double)nt * nt * nt);
        ns = per_tile > 64 ? 4 : (per_tile > 8 ? 3 : 2);
    }
    while (ns > 1 && (double)nt * ns * nt * ns * nt * ns > 2.0e9) --ns;
    return ns;
}

Geom make_geom(double box, double x_s, double r_cut, int nt, int ns, double eps_b) {
    Geom g{};
    g.box = box;
    g.inv_box = 1.0 / box;
    g.rc2 = r_cut * r_cut;
    g.nt = nt;
    g.ns = ns;
    g.nc = nt * ns;
    g.ns3 = ns * ns * ns;
    g.nt3 = nt * nt * nt;
    g.tile = box / nt;
    g.sub = g.tile / ns;
    g.inv_cell = (double)g.nc / box;
    double margin = r_cut * 1e-9 + box * 1e-12;
    g.cull2 = (r_cut + margin) * (r_cut + margin);
    g.x_s = x_s;
    g.k1 = 1.0 / (2.0 * x_s);
    g.k2 = -1.4426950408889634074 / (4.0 * x_s * x_s);
    g.kb = 1.0 / (2.0 * 1.77245385090551602730 * x_s * x_s * x_s);
    g.k1f = (float)g.k1;
    g.kbf = (float)g.kb;
    g.c2 = 1.0 / (4.0 * x_s * x_s);
    g.c3 = 1.0 / (8.0 * x_s * x_s * x_s);
    g.c2f = (float)g.c2;
    g.c3f = (float)g.c3;
    static_assert(P3M_H64_DEGREE + 1 <= (int)(sizeof(g.h64) / sizeof(double)), "H64 table");
    for (int k = 0; k <= P3M_H64_DEGREE; ++k) g.h64[k] = kH64[k];
    if (eps_b > 0.0) {
        g.eps_b = eps_b;
        g.eps_b2 = eps_b * eps_b;
        g.inv_eps_b = 1.0 / eps_b;
        g.ks3 = 32.0 / (eps_b * eps_b * eps_b);
        g.ks5 = g.ks3 / (eps_b * eps_b);
        g.inv_eps_bf = (float)g.inv_eps_b;
    }
    return g;
}

struct Request {
    const double *pos;
    const double *mass;
    const uint8_t *sel;      // active mask or rung
    int sel_kind;            // SelKind for receivers
    int n_sub;
    const uint8_t *thr;      // host thresholds (rung mode)
    int64_t n;
    double box, x_s, r_cut;
    int precision;
    bool backward;
    const double *grad_acc;
    double *out;
    hipStream_t stream;
    int force_ns;            // >0: override subtiles (autotune trials)
    int force_target;
    int force_csize;         // >0: override the cluster size
    int force_screen;        // 0: not forced, 1: screening off, 2: on
};

// Default layout before tuning: full 64-receiver clusters without screening.
constexpr int kDefaultCsize = 64;
constexpr int kDefaultScreen = 0;
// screen == kScreenMutual: all-active FP32 forward calls evaluate each pair
// once for both partners (other calls screen)
constexpr int kScreenMutual = 2;

bool valid_csize(int c) { return c == 8 || c == 16 || c == 32 || c == 64; }

// B-spline softening length per Plummer-equivalent one (section 2.1.1, below
// eq. bspline_force: eps_B = 2.8 eps).
constexpr double kBsplinePerPlummer = 2.8;

int run(p3m_sr_context *h, const Request &r, SrWork &w) {
    hipStream_t s = r.stream;
    const int n = (int)r.n;
    const bool fp32 = r.precision == P3M_FP32;
    const int n_sub = r.n_sub;
    const int nt = tiles_per_dim(r.box, r.r_cut);

    const double eps_b = kBsplinePerPlummer * h->eps;
    // one subset with every particle a receiver: receivers are the sorted
    // particles themselves, no flags, scan or compaction
    const bool all_recv = n_sub == 1 && (r.backward || r.sel_kind == SEL_ALL);
    // tabulated FP32 shape (point particles, forward only)
    const int shape = (fp32 && !r.backward && eps_b == 0.0) ? h->cfg_shape : SHAPE_POLY;
    // each pair once for both partners: calls with every particle a receiver
    // (all-active forward calls with the polynomial shape, softened or not,
    // and the adjoint without softening, in both precisions), fewer than 2^27
    // particles
    // (the list entries hold the sorted index in 27 bits), not in the
    // deterministic mode (its reactions are added with atomics), and
    // clusters of 16, 32 or 64
    const bool det = h->deterministic;
    const bool mutual_ok = all_recv && shape == SHAPE_POLY &&
                           (eps_b == 0.0 || !r.backward) &&
                           r.n <= (int64_t)(1u << 27) && !det;

    // decomposition: explicit override > user config > autotuned > default
    int ns = 0, target = 0, csize = 0, screen = -1;
    const int mode = (r.backward ? 2 : 0) + (fp32 ? 0 : 1);
    const int tkind = r.backward ? TUNE_ADJOINT
                                 : (r.sel_kind == SEL_RUNG ? TUNE_BATCHED : TUNE_FORWARD);
    auto it = h->tuned.find(TuneKey{r.n, nt, r.precision, tkind, tkind == TUNE_BATCHED ? n_sub : 1});
    // a rung-batched call not tuned on its own takes the forward's layout
    if (it == h->tuned.end() && tkind == TUNE_BATCHED)
        it = h->tuned.find(TuneKey{r.n, nt, r.precision, TUNE_FORWARD, 1});
    // a tuned layout that pairs once for both partners, on a call that
    // cannot: the fastest of the other layouts, where one was kept
    if (it != h->tuned.end() && it->second.screen == kScreenMutual && !mutual_ok) {
        const int pk = plain_kind(it->first.kind);
        auto p = pk < 0 ? h->tuned.end() : h->tuned.find(TuneKey{r.n, nt, r.precision, pk, 1});
        if (p != h->tuned.end()) it = p;
    }
    if (it != h->tuned.end()) {
        ns = it->second.ns;
        target = it->second.target;
        csize = it->second.csize;
        screen = it->second.screen;
    }
    if (h->cfg_ns > 0) ns = h->cfg_ns;
    if (h->cfg_target > 0) target = h->cfg_target;
    if (h->cfg_csize > 0) csize = h->cfg_csize;
    if (h->cfg_screen >= 0) screen = h->cfg_screen;
    if (r.force_ns > 0) ns = r.force_ns;
    if (r.force_target > 0) target = r.force_target;
    if (r.force_csize > 0) csize = r.force_csize;
    if (r.force_screen > 0) screen = r.force_screen - 1;
    ns = pick_subtiles(nt, r.n, ns);
    if (target <= 0) target = 1024;
    if (!valid_csize(csize)) csize = kDefaultCsize;
    if (screen < 0) screen = kDefaultScreen;
    const Geom g = make_geom(r.box, r.x_s, r.r_cut, nt, ns, eps_b);
    const size_t ncells = (size_t)g.nt3 * g.ns3;
    // other calls with this layout take the screened kernel
    const bool mutual = screen == kScreenMutual && mutual_ok && csize >= 16;
    if (screen == kScreenMutual && !mutual) screen = 1;

    p3m_sr_stats st{};
    st.n = r.n;
    st.tiles_per_dim = nt;
    st.subtiles_per_dim = ns;
    st.item_target = target;
    st.precision = r.precision;
    st.cluster_size = csize;
    st.screen = mutual ? kScreenMutual : screen;
    st.deterministic = det ? 1 : 0;
    st.eps_b = kBsplinePerPlummer * h->eps;
    st.ms_build = st.ms_pairs = st.ms_total = st.ms_sort = -1.0f;
    h->last_stream = s;
    h->timed_last = false;
    h->sort_b = false;
    if (h->timing) P3M_HIP(hipEventRecord(h->ev[0], s));

    const size_t out_elems = (size_t)n_sub * (size_t)n * 3;
    if (n == 0) {
        h->stats = st;
        return P3M_OK;
    }

    // ---- workspace (every buffer is taken before the first launch, apart
    // from the work items, whose count the device reports) ----
    w.used = 0;
    const size_t nflags = (size_t)n * n_sub;
    const size_t ncl_len = (size_t)n_sub * g.nt3;
    const size_t cl_bound = ncl_len + (nflags + csize - 1) / csize;
    const size_t det_hist = det ? stable_rank_hist_ints(n) : 0;
    const size_t scan_max = std::max(std::max(std::max(ncells, nflags), std::max(ncl_len, cl_bound)),
                                     det_hist);
    int rc;
    if ((rc = take(h, w, w.key, sizeof(int) * n, s))) return rc;
    if ((rc = take(h, w, w.rank, sizeof(int) * n, s))) return rc;
    if ((rc = take(h, w, w.cells, sizeof(int) * (ncells + 1), s))) return rc;
    if ((rc = take(h, w, w.fbig, sizeof(int) * (2 + (size_t)n / kFineBig), s))) return rc;
    if ((rc = take(h, w, w.sp, sizeof(double4) * ((size_t)n + kSupplierPad), s))) return rc;
    if ((rc = take(h, w, w.perm, sizeof(int) * n, s))) return rc;
    if ((rc = take(h, w, w.sel, (size_t)n, s))) return rc;
    if ((rc = take(h, w, w.sp2, sizeof(double4) * ((size_t)n + kSupplierPad), s))) return rc;
    if ((rc = take(h, w, w.perm2, sizeof(int) * n, s))) return rc;
    if ((rc = take(h, w, w.sel2, (size_t)n, s))) return rc;
    if ((rc = take(h, w, w.flags, sizeof(int) * (nflags + 1), s))) return rc;
    if ((rc = take(h, w, w.actpos, sizeof(int) * (nflags + 1), s))) return rc;
    if ((rc = take(h, w, w.ncl, sizeof(int) * (ncl_len + 1), s))) return rc;
    if ((rc = take(h, w, w.clusters, sizeof(Cluster) * cl_bound, s))) return rc;
    if ((rc = take(h, w, w.itemcnt, sizeof(int) * (cl_bound + 1), s))) return rc;
    if ((rc = take(h, w, w.bsum, sizeof(int) * scan_block_sums_needed(scan_max), s))) return rc;
    if ((rc = take(h, w, w.counters, sizeof(Counters) * kCounterCopies * kCounterStride, s)))
        return rc;
    if ((rc = take(h, w, w.scal, sizeof(int) * kXcds * kQueueStride, s))) return rc;
    if ((rc = take(h, w, w.rp, sizeof(double4) * (nflags + 1), s))) return rc;
    if ((rc = take(h, w, w.rperm, sizeof(int) * (nflags + 1), s))) return rc;
    if (r.backward && (rc = take(h, w, w.rwa, sizeof(double4) * (nflags + 1), s))) return rc;
    if (r.backward && (rc = take(h, w, w.wa, sizeof(double4) * ((size_t)n + kSupplierPad), s))) return rc;
    if (mutual && (rc = take(h, w, w.msum, sizeof(double) * 3 * (size_t)n, s))) return rc;
    // the call's single-pass scans (cells, receiver flags, clusters, items)
    const size_t s1_cells = scan1_status_needed(ncells);
    const size_t s1_flags = all_recv ? 0 : scan1_status_needed(nflags);
    const size_t s1_ncl = scan1_status_needed(ncl_len);
    const size_t s1_items = scan1_status_needed(cl_bound);
    const size_t s1_total = s1_cells + s1_flags + s1_ncl + s1_items;
    if ((rc = take(h, w, w.scan1, sizeof(unsigned long long) * s1_total + 4 * sizeof(int), s)))
        return rc;
    if (det) {
        if ((rc = take(h, w, w.det_k, sizeof(unsigned long long) * 2 * (size_t)n, s))) return rc;
        if ((rc = take(h, w, w.det_v, sizeof(int) * 2 * (size_t)n, s))) return rc;
        if ((rc = take(h, w, w.det_hist, sizeof(int) * (det_hist + 1), s))) return rc;
    }
    if (shape != SHAPE_POLY && (rc = take(h, w, w.htab, kTabFloats * sizeof(float), s)))
        return rc;
    // work items: the array is sized by the bound on their count (plan_items
    // gives a cluster at most plan_items_bound), so the host never waits for
    // the count, unless that bound passes kItemBoundBytes (or what is left of
    // the fixed workspace), or in the deterministic mode, whose partial slots
    // are per item: then the host waits for the count (below)
    const size_t item_bound = cl_bound * (size_t)plan_items_bound(g.ns3, mutual ? 1 : 0);
    bool wait_count = det || item_bound * sizeof(Item) > kItemBoundBytes ||
                      item_bound > (size_t)INT_MAX;
    if (!wait_count && w.base && w.used + item_bound * sizeof(Item) + 256 > w.size)
        wait_count = true;
    if (!wait_count && (rc = take(h, w, w.items, sizeof(Item) * item_bound, s))) return rc;
    // With every particle a receiver the clusters and items follow from the
    // cell counts alone (a cluster is a run of consecutive sorted particles
    // of one subtile, whatever their order inside it): their planning runs
    // on its own stream beside the scatter and the fine order, and only the
    // cluster boxes, which read the final order, wait for both.
    const bool early_plan = all_recv && !det && !wait_count;

    int *key = (int *)w.key.p, *rank = (int *)w.rank.p, *cells = (int *)w.cells.p;
    double4 *sp = (double4 *)w.sp.p;
    int *perm = (int *)w.perm.p;
    uint8_t *sel_s = (uint8_t *)w.sel.p;
    int *flags = (int *)w.flags.p, *actpos = (int *)w.actpos.p, *ncl = (int *)w.ncl.p;
    Cluster *clusters = (Cluster *)w.clusters.p;
    int *itemcnt = (int *)w.itemcnt.p, *bsum = (int *)w.bsum.p;
    Counters *counters = (Counters *)w.counters.p;
    h->last_counters = counters;
    int *scal = (int *)w.scal.p;   // the XCD work queues, kQueueStride ints apart

    // ---- sort ----
    int *fbig = (int *)w.fbig.p;
    int *queue = scal;
    double4 *sp_f = (double4 *)w.sp2.p;   // the sorted particles after the fine order
    {
        // every small initialisation of the call in one launch
        FillSet f{};
        f.add(cells, ncells + 1, 0);
        f.add((int *)counters, sizeof(Counters) * kCounterCopies * kCounterStride / sizeof(int), 0);
        f.add(fbig, 1, 0);
        f.add(queue, kXcds * kQueueStride, 0);
        f.add((int *)(sp_f + n), kSupplierPad * sizeof(double4) / sizeof(int), 0);
        if (all_recv) f.add(flags + nflags, 1, n);   // the receiver total
        f.add((int *)w.scan1.p, 2 * s1_total + 4, 0);
        P3M_HIP(launch_fill_multi(f, s));
    }
    unsigned long long *s1 = (unsigned long long *)w.scan1.p;
    int *s1c = (int *)(s1 + s1_total);
    unsigned long long *stall = &counters->scan_stall;
    P3M_HIP(launch_keys(r.pos, n, g, key, rank, cells, s));
    P3M_HIP(launch_scan1(cells, cells, ncells, s1, s1c, stall, bsum, s));
    if (early_plan) {
        P3M_HIP(hipEventRecord(h->pfork, s));
        P3M_HIP(hipStreamWaitEvent(h->pstream, h->pfork, 0));
        hipStream_t ps = h->pstream;
        P3M_HIP(launch_cluster_count(cells, nullptr, n, n_sub, g, csize, ncl, ps));
        P3M_HIP(launch_scan1(ncl, ncl, ncl_len, s1 + s1_cells + s1_flags, s1c + 2, stall, bsum, ps));
        P3M_HIP(launch_cluster_write(cells, nullptr, ncl, n, n_sub, g, csize, clusters, ps));
        P3M_HIP(launch_item_count(clusters, ncl + ncl_len, (int)cl_bound, cells, g, target,
                                  mutual ? 1 : 0, itemcnt, ps));
        P3M_HIP(launch_scan1(itemcnt, itemcnt, cl_bound, s1 + s1_cells + s1_flags + s1_ncl,
                             s1c + 3, stall, bsum, ps));
        P3M_HIP(launch_item_write(clusters, ncl + ncl_len, (int)cl_bound, cells, g, target,
                                  mutual ? 1 : 0, itemcnt, (Item *)w.items.p, flags + nflags,
                                  itemcnt + cl_bound, h->host_tot, ps));
        if (shape != SHAPE_POLY)
            P3M_HIP(launch_build_htab(shape, h->cfg_tab_n, g, (float *)w.htab.p, ps));
        P3M_HIP(hipEventRecord(h->pjoin, ps));
        // the dense subtiles' list needs only the cell counts as well
        P3M_HIP(hipStreamWaitEvent(h->bstream, h->pfork, 0));
        P3M_HIP(launch_big_list(cells, g, fbig, h->bstream));
    }
    if (det) {
        // ranks in (fine sub-cell, index) order instead of the atomics' order
        unsigned long long *k64 = (unsigned long long *)w.det_k.p;
        int *v = (int *)w.det_v.p;
        P3M_HIP(launch_stable_ranks(r.pos, n, g, key, cells, k64, k64 + n, v, v + n,
                                    (int *)w.det_hist.p, bsum, rank, s));
    }
    const uint8_t *sel_src = (r.sel_kind == SEL_ALL && !r.backward) ? nullptr : r.sel;
    {
        int *perm_f = (int *)w.perm2.p;
        uint8_t *sel_f = (uint8_t *)w.sel2.p;
        // without a selector the selector arrays stay unwritten (nullptr):
        // the later kernels then take every particle as active
        if (!sel_src) sel_s = sel_f = nullptr;
        P3M_HIP(launch_scatter(r.pos, r.mass, sel_src, n, g, key, rank, cells, fp32 ? 1 : 0,
                               csize, det, sp, perm, sel_s, sp_f, perm_f, sel_f, s));
        // fine order inside dense subtiles (key/rank are free again as scratch)
        // a subtile no larger than one cluster gains nothing from the reorder;
        // the stable ranks are in fine order already.  The subtiles above
        // kFineBig particles are ordered on the build stream meanwhile (the
        // box kernel needs both orders).
        if (!det) {
            if (!early_plan) P3M_HIP(launch_big_list(cells, g, fbig, s));
            P3M_HIP(hipEventRecord(h->bsort, s));
            P3M_HIP(hipStreamWaitEvent(h->bstream, h->bsort, 0));
            P3M_HIP(launch_fine_order_big(sp, perm, sel_s, cells, g, key, rank, sp_f, perm_f,
                                          sel_f, n, fbig, h->bstream));
            if (h->timing) P3M_HIP(hipEventRecord(h->ev[5], h->bstream));
            h->sort_b = h->timing;
            // the receiver flags read the final selectors, the dense
            // subtiles' among them: with flags the call's stream waits here
            if (!all_recv) P3M_HIP(hipEventRecord(h->bsorted, h->bstream));
            // the output (the mutual kernel: its sorted-order sums) is cleared
            // on the build stream meanwhile; nothing before the pair kernel
            // reads it
            if (mutual) P3M_HIP(launch_fill_f64((double *)w.msum.p, 0.0, 3 * (size_t)n, h->bstream));
            else P3M_HIP(launch_fill_f64(r.out, 0.0, out_elems, h->bstream));
            // with the early planning the cluster boxes wait here: they read
            // the final order (and the pair kernel the cleared output)
            if (early_plan) P3M_HIP(hipEventRecord(h->bsorted, h->bstream));
            P3M_HIP(launch_fine_order_medium(sp, perm, sel_s, cells, g, key, rank, sp_f, perm_f,
                                             sel_f, csize, s));
        }
        sp = sp_f;
        perm = perm_f;
        sel_s = sel_f;
    }
    if (h->timing) P3M_HIP(hipEventRecord(h->ev[4], s));

    // ---- receivers -> clusters -> items ----
    // the adjoint needs every particle as a receiver (its output rows are
    // the particles near any active one); activity enters through wa
    const int kind = r.backward ? SEL_ALL : r.sel_kind;
    const int *recv_scan = flags, *recv_pos = actpos;
    double4 *wa = r.backward ? (double4 *)w.wa.p : nullptr;
    // receivers, clusters and items reach the stats when they are asked for
    st.receivers = st.clusters = st.items = -1;
    if (early_plan) {
        // the clusters and items are planned on their own stream already;
        // the boxes wait for both halves of the fine order and for the
        // planning, which is then also done before the pair kernel
        P3M_HIP(hipStreamWaitEvent(s, h->bsorted, 0));
        P3M_HIP(hipStreamWaitEvent(s, h->pjoin, 0));
        if (r.backward) P3M_HIP(launch_gather_weights(r.grad_acc, sel_s, perm, n, fp32, wa, s));
        P3M_HIP(launch_cluster_finish(clusters, ncl + ncl_len, cl_bound, csize, nullptr, sp, perm,
                                      wa, nullptr, nullptr, nullptr, s));
    } else {
        if (all_recv) {
            recv_scan = recv_pos = nullptr;
        } else {
            if (!det) P3M_HIP(hipStreamWaitEvent(s, h->bsorted, 0));
            P3M_HIP(launch_flags(sel_s, n, n_sub, kind, r.thr, flags, s));
            P3M_HIP(launch_scan1(flags, flags, nflags, s1 + s1_cells, s1c + 1, stall, bsum, s));
            P3M_HIP(launch_compact(flags, n, n_sub, actpos, s));
        }
        P3M_HIP(launch_cluster_count(cells, recv_scan, n, n_sub, g, csize, ncl, s));
        P3M_HIP(launch_scan1(ncl, ncl, ncl_len, s1 + s1_cells + s1_flags, s1c + 2, stall, bsum, s));
        P3M_HIP(launch_cluster_write(cells, recv_scan, ncl, n, n_sub, g, csize, clusters, s));

        // The cluster boxes, the receiver gather, the table (and in the
        // deterministic mode the output clear) need neither each other's
        // results nor the item planning: they run on the build stream beside
        // it, joined before the pair kernel.  (The box kernel writes only the
        // boxes of the cluster records, the item kernels read only the other
        // fields.)
        P3M_HIP(hipEventRecord(h->bfork, s));
        P3M_HIP(hipStreamWaitEvent(h->bstream, h->bfork, 0));
        hipStream_t bs = h->bstream;
        if (r.backward) P3M_HIP(launch_gather_weights(r.grad_acc, sel_s, perm, n, fp32, wa, bs));
        // with every particle a receiver the receivers are sp / perm / wa as they are
        double4 *rp = all_recv ? nullptr : (double4 *)w.rp.p;
        P3M_HIP(launch_cluster_finish(clusters, ncl + ncl_len, cl_bound, csize, recv_pos, sp, perm,
                                      wa, rp, (int *)w.rperm.p,
                                      r.backward ? (double4 *)w.rwa.p : nullptr, bs));
        // the output is cleared here in the deterministic mode (which has no
        // mutual kernel), else on the build stream beside the fine order
        if (det) P3M_HIP(launch_fill_f64(r.out, 0.0, out_elems, bs));
        if (shape != SHAPE_POLY)
            P3M_HIP(launch_build_htab(shape, h->cfg_tab_n, g, (float *)w.htab.p, bs));
        P3M_HIP(hipEventRecord(h->bjoin, bs));

        P3M_HIP(launch_item_count(clusters, ncl + ncl_len, (int)cl_bound, cells, g, target,
                                  mutual ? 1 : 0, itemcnt, s));
        P3M_HIP(launch_scan1(itemcnt, itemcnt, cl_bound, s1 + s1_cells + s1_flags + s1_ncl,
                             s1c + 3, stall, bsum, s));
        // the three totals go to pinned memory for the stats: here when the
        // call waits for the item count, else from the item writer
        if (wait_count) {
            P3M_HIP(launch_totals(flags + nflags, ncl + ncl_len, itemcnt + cl_bound, h->host_tot,
                                  s));
            P3M_HIP(hipEventRecord(h->tot_ev, s));
            P3M_HIP(hipEventSynchronize(h->tot_ev));
            const size_t n_items = (size_t)std::max(h->host_tot[2], 1);
            if ((rc = take(h, w, w.items, sizeof(Item) * n_items, s))) return rc;
            if (det &&
                (rc = take(h, w, w.partials, sizeof(double) * 3 * (size_t)csize * n_items, s)))
                return rc;
        }
        // the totals for the stats (already there when the call waited for them)
        P3M_HIP(launch_item_write(clusters, ncl + ncl_len, (int)cl_bound, cells, g, target,
                                  mutual ? 1 : 0, itemcnt, (Item *)w.items.p, flags + nflags,
                                  itemcnt + cl_bound, wait_count ? nullptr : h->host_tot, s));
        P3M_HIP(hipStreamWaitEvent(s, h->bjoin, 0));
    }
    Item *items = (Item *)w.items.p;

    // ---- pairs ----
    PairArgs a{};
    a.sp = sp;
    a.rp = all_recv ? sp : (const double4 *)w.rp.p;
    a.rwa = all_recv ? wa : (const double4 *)w.rwa.p;
    a.cell_start = cells;
    a.clusters = clusters;
    a.items = items;
    a.wa = wa;
    a.queue = queue;
    a.rperm = all_recv ? perm : (const int *)w.rperm.p;
    a.out = r.out;
    a.out_stride = 3ll * n;
    a.counters = counters;
    a.n_items_dev = itemcnt + cl_bound;
    a.partials = det ? (double *)w.partials.p : nullptr;
    a.unit_mass = r.mass ? 0 : 1;
    a.csize = csize;
    a.g = g;
    if (shape != SHAPE_POLY) {
        a.htab = (const float *)w.htab.p;
        a.tab_n = h->cfg_tab_n;
        a.tab_scale = (float)((double)h->cfg_tab_n / g.rc2);
    }
    st.shape = shape;
    const int unit = r.mass ? 0 : 1, soft = g.eps_b > 0.0 ? 1 : 0;
    const int cs_idx = csize == 8 ? 0 : csize == 16 ? 1 : csize == 32 ? 2 : 3;
    int bpc;
    if (mutual) {
        int &slot_m =
            h->mutual_blocks_per_cu[(((cs_idx * 2 + (r.backward ? 1 : 0)) * 2 + unit) * 2 + soft) * 2 +
                                    (fp32 ? 0 : 1)];
        if (slot_m == 0) slot_m = mutual_blocks_per_cu(csize, unit, r.backward, soft != 0, !fp32);
        bpc = slot_m;
        a.out = (double *)w.msum.p;
        a.out_stride = n;
        a.rc2_lo = (float)(g.rc2 * (1.0 - std::ldexp(1.0, -17)));
        a.rc2_hi = (float)(g.rc2 * (1.0 + std::ldexp(1.0, -17)));
    } else {
        const int slot =
            (((mode * 2 + (screen ? 1 : 0)) * 4 + cs_idx) * 3 + shape) * 4 + unit * 2 + soft;
        int &slot_b = h->blocks_per_cu[slot];
        if (slot_b == 0) slot_b = pairs_blocks_per_cu(mode, screen, shape, csize, unit, soft);
        bpc = slot_b;
    }
    // every resident block (the kernels read the item count and size their
    // queue claims on the device; blocks without work leave at once)
    long long grid = (long long)h->n_cu * bpc;
    if (grid < 1) grid = 1;
    if (h->timing) P3M_HIP(hipEventRecord(h->ev[1], s));
    if (mutual) P3M_HIP(launch_pairs_mutual(a, r.backward, !fp32, (int)grid, s));
    else P3M_HIP(launch_pairs(mode, screen, shape, a, (int)grid, s));
    if (mutual) P3M_HIP(launch_mutual_out((const double *)w.msum.p, perm, n, r.out, s));
    if (det)
        P3M_HIP(launch_item_reduce(clusters, ncl + ncl_len, (int)cl_bound, itemcnt, a.partials,
                                   csize, a.rperm, r.out, a.out_stride, s));
    if (h->timing) {
        P3M_HIP(hipEventRecord(h->ev[2], s));
        h->timed_last = true;
    }
    if (h->timing) P3M_HIP(hipEventRecord(h->ev[3], s));
    h->stats = st;
    return P3M_OK;
}

int check_handle(p3m_sr_handle h) {
    if (!h) return set_error(P3M_EINVAL, "NULL handle");
    return P3M_OK;
}

int set_device(p3m_sr_handle h) {
    int cur = -1;
    P3M_HIP(hipGetDevice(&cur));
    if (cur != h->device) P3M_HIP(hipSetDevice(h->device));
    return P3M_OK;
}

// The long-range call after its arguments were checked (also used by the
// KDK step).
int lr_run(p3m_sr_context *h, const double *pos, const double *mass, const uint8_t *active,
           int np, double box, int n_grid, double x_s, double *acc_out, hipStream_t s) {
    int rc;
    const size_t g = (size_t)n_grid;
    const size_t nh = ((g / 2 + 1) + 7) & ~(size_t)7;   // padded half-spectrum row
    if ((rc = ensure(h, h->pm_real, g * g * g * sizeof(double), s))) return rc;
    if ((rc = ensure(h, h->pm_spec, nh * g * g * 2 * sizeof(double), s))) return rc;
    if ((rc = ensure(h, h->pm_tab, (g / 2) * 2 * sizeof(double) + 2 * g * sizeof(double), s)))
        return rc;
    const size_t cells = g * g * g;
    const size_t np1 = (size_t)np + 1;
    if ((rc = ensure(h, h->pm_cnt, (cells + 1) * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->pm_bsum, sizeof(int) * scan_block_sums_needed(cells), s))) return rc;
    if ((rc = ensure(h, h->pm_key, np1 * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->pm_rank, np1 * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->pm_rec, np1 * sizeof(double4), s))) return rc;
    if ((rc = ensure(h, h->pm_nkey, np1 * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->pm_perm, np1 * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->pm_recv, np1, s))) return rc;
    h->last_stream = s;
    double2 *tw = (double2 *)h->pm_tab.p;
    double *w1 = (double *)(tw + g / 2);
    double *k2 = w1 + g;
    const double hcell = box / (double)n_grid;
    const bool timing = h->timing;
    if (timing) {
        for (hipEvent_t &e : h->lr_ev)
            if (!e) P3M_HIP(hipEventCreate(&e));
        P3M_HIP(hipEventRecord(h->lr_ev[0], s));
    }
    double4 *rec = (double4 *)h->pm_rec.p;
    int *nkey = (int *)h->pm_nkey.p, *perm = (int *)h->pm_perm.p;
    uint8_t *recv = (uint8_t *)h->pm_recv.p;
    P3M_HIP(launch_pm_tables(n_grid, box, x_s, tw, w1, k2, s));
    P3M_HIP(launch_pm_sort(pos, mass, active, np, n_grid, box, hcell, (int *)h->pm_key.p,
                           (int *)h->pm_rank.p, (int *)h->pm_cnt.p, (int *)h->pm_bsum.p, rec, nkey,
                           perm, recv, s));
    if (timing) P3M_HIP(hipEventRecord(h->lr_ev[1], s));
    P3M_HIP(launch_pm_deposit(rec, nkey, (const int *)h->pm_cnt.p, np, (double *)h->pm_real.p,
                              n_grid, s));
    if (timing) P3M_HIP(hipEventRecord(h->lr_ev[2], s));
    PmArgs a{};
    a.n = n_grid;
    a.real = (double *)h->pm_real.p;
    a.spec = (double2 *)h->pm_spec.p;
    a.tw = tw;
    a.w1 = w1;
    a.k2 = k2;
    a.scale = 4.0 * M_PI / (hcell * hcell * hcell * hcell) / ((double)g * (double)g * (double)g);
    P3M_HIP(launch_pm_fft_chain(a, s, timing ? h->lr_ev + 3 : nullptr));
    if (timing) P3M_HIP(hipEventRecord(h->lr_ev[7], s));
    P3M_HIP(launch_pm_readout(rec, nkey, perm, recv, np, (const double *)h->pm_real.p, n_grid,
                              acc_out, s));
    if (timing) P3M_HIP(hipEventRecord(h->lr_ev[8], s));
    h->lr_stats = p3m_lr_stats{};
    h->lr_stats.n = np;
    h->lr_stats.n_grid = n_grid;
    h->lr_timed = timing;
    h->lr_stream = s;
    return P3M_OK;
}

}  // namespace

extern "C" {

const char *p3m_sr_last_error(void) { return g_last_error.c_str(); }

const char *p3m_sr_version(void) { return "p3msr 0.1 (gfx950)"; }

int p3m_sr_create(p3m_sr_handle *out, int device) {
    if (!out) return set_error(P3M_EINVAL, "NULL output pointer");
    *out = nullptr;
    int ndev = 0;
    P3M_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return set_error(P3M_EINVAL, "device %d out of range (%d devices)", device, ndev);
    P3M_HIP(hipSetDevice(device));
    p3m_sr_context *h = new p3m_sr_context();
    h->device = device;
    // fine-grained (coherent) pinned memory: the kernel's stores reach the
    // host without a cache flush, and are read after the stream synchronises
    if (hipHostMalloc((void **)&h->host_tot, 4 * sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return set_error(P3M_ENOMEM, "pinned host scalars could not be allocated");
    }
    if (hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        h->n_cu <= 0)
        h->n_cu = 256;
    // the fixed workspace of the no-alloc entry point on this device
    {
        void *base = nullptr;
        const int rc = scratch_address(device, &base);
        if (rc) {
            p3m_sr_destroy(h);
            return rc;
        }
        h->fixed.base = (unsigned char *)base;
        h->fixed.size = kNoAllocBytes;
    }
    // the autotuner's persistent cache
    h->device_id = device_identity(device);
    h->cache_path = default_cache_path();
    load_cache(h);
    // the events every call may record (timing, the totals' arrival)
    bool ev_ok = hipEventCreateWithFlags(&h->tot_ev, hipEventDisableTiming) == hipSuccess;
    for (hipEvent_t &e : h->ev) ev_ok = ev_ok && hipEventCreate(&e) == hipSuccess;
    ev_ok = ev_ok && hipEventCreateWithFlags(&h->bfork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->bsort, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->bsorted, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->bjoin, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&h->bstream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&h->pfork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->pjoin, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&h->pstream, hipStreamNonBlocking) == hipSuccess;
    if (!ev_ok) {
        (void)hipGetLastError();
        p3m_sr_destroy(h);
        return set_error(P3M_EHIP, "events could not be created");
    }
    *out = h;
    return P3M_OK;
}

int p3m_sr_destroy(p3m_sr_handle h) {
    if (!h) return P3M_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    SrWork &w = h->work;
    DevBuf *bufs[] = {&w.key,     &w.rank,     &w.cells,    &w.sp,      &w.perm,
                      &w.sel,     &w.sp2,      &w.perm2,    &w.sel2,    &w.flags,
                      &w.actpos,  &w.ncl,      &w.clusters, &w.itemcnt, &w.items,
                      &w.bsum,    &w.counters, &w.wa,       &w.scal,    &w.rp,
                      &w.rperm,   &w.rwa,      &w.fbig,     &w.msum,    &w.htab,
                      &w.det_k,   &w.det_v,    &w.det_hist, &w.partials, &w.scan1,
                      &h->pm_real, &h->pm_spec, &h->pm_tab, &h->pm_key,  &h->pm_rank,
                      &h->pm_cnt,  &h->pm_rec,  &h->pm_nkey, &h->pm_perm, &h->pm_recv,
                      &h->kdk_acc, &h->kdk_lr,  &h->kdk_tq,  &h->kdk_tnext, &h->kdk_due,
                      &h->kdk_scal, &h->pm_bsum, &h->p3m_lr, &h->tune_w, &h->tune_sig};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (hipEvent_t e : h->ev)
        if (e) (void)hipEventDestroy(e);
    if (h->tot_ev) (void)hipEventDestroy(h->tot_ev);
    for (hipEvent_t e : h->lr_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->host_tot) (void)hipHostFree(h->host_tot);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
    if (h->aux) (void)hipStreamDestroy(h->aux);
    if (h->bfork) (void)hipEventDestroy(h->bfork);
    if (h->bsort) (void)hipEventDestroy(h->bsort);
    if (h->bsorted) (void)hipEventDestroy(h->bsorted);
    if (h->bjoin) (void)hipEventDestroy(h->bjoin);
    if (h->bstream) (void)hipStreamDestroy(h->bstream);
    if (h->pfork) (void)hipEventDestroy(h->pfork);
    if (h->pjoin) (void)hipEventDestroy(h->pjoin);
    if (h->pstream) (void)hipStreamDestroy(h->pstream);
    delete h;
    return P3M_OK;
}

int p3m_sr_force(p3m_sr_handle h, const double *pos, const double *mass, const uint8_t *active,
                 int64_t n, double box, double x_s, double r_cut, int precision, double *acc_out,
                 void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    if (n > 0 && (!pos || !acc_out)) return set_error(P3M_EINVAL, "pos and acc_out are required");
    if (!aligned8(pos) || !aligned8(acc_out) || !aligned8(mass))
        return set_error(P3M_EINVAL, "pos, mass and acc_out must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if ((rc = set_device(h))) return rc;
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = active;
    r.sel_kind = active ? SEL_MASK : SEL_ALL;
    r.n_sub = 1;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc_out;
    r.stream = (hipStream_t)stream;
    return run(h, r, h->work);
}

int p3m_sr_force_noalloc(p3m_sr_handle h, const double *pos, const double *mass,
                         const uint8_t *active, int64_t n, double box, double x_s, double r_cut,
                         int precision, double *acc_out, void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    if (n > 0 && (!pos || !acc_out)) return set_error(P3M_EINVAL, "pos and acc_out are required");
    if (!aligned8(pos) || !aligned8(acc_out) || !aligned8(mass))
        return set_error(P3M_EINVAL, "pos, mass and acc_out must be 8-byte aligned");
    if (n > kNoAllocMaxN)
        return set_error(P3M_EUNSUPPORTED,
                         "n = %lld exceeds the no-alloc limit of %lld particles", (long long)n,
                         (long long)kNoAllocMaxN);
    if ((rc = check_handle(h))) return rc;
    if (!h->fixed.base) return set_error(P3M_EHIP, "the no-alloc workspace is not available");
    if ((rc = set_device(h))) return rc;
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = active;
    r.sel_kind = active ? SEL_MASK : SEL_ALL;
    r.n_sub = 1;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc_out;
    r.stream = (hipStream_t)stream;
    return run(h, r, h->fixed);
}

int p3m_sr_force_backward(p3m_sr_handle h, const double *pos, const double *mass,
                          const uint8_t *active, int64_t n, double box, double x_s, double r_cut,
                          int precision, const double *grad_acc, double *grad_pos,
                          void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    if (n > 0 && (!pos || !grad_acc || !grad_pos))
        return set_error(P3M_EINVAL, "pos, grad_acc and grad_pos are required");
    if (!aligned8(pos) || !aligned8(mass) || !aligned8(grad_acc) || !aligned8(grad_pos))
        return set_error(P3M_EINVAL, "pos, mass, grad_acc and grad_pos must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if ((rc = set_device(h))) return rc;
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = active;
    r.sel_kind = active ? SEL_MASK : SEL_ALL;
    r.n_sub = 1;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.backward = true;
    r.grad_acc = grad_acc;
    r.out = grad_pos;
    r.stream = (hipStream_t)stream;
    return run(h, r, h->work);
}

int p3m_sr_force_batched(p3m_sr_handle h, const double *pos, const double *mass,
                         const uint8_t *rung, int64_t n, int n_sub, const uint8_t *min_rung,
                         double box, double x_s, double r_cut, int precision, double *acc_out,
                         void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    if (n_sub < 1 || n_sub > 64) return set_error(P3M_EINVAL, "n_sub must be in 1..64");
    if (!min_rung) return set_error(P3M_EINVAL, "min_rung (host array) is required");
    if (n > 0 && (!pos || !rung || !acc_out))
        return set_error(P3M_EINVAL, "pos, rung and acc_out are required");
    if ((double)n * n_sub > 2.0e9)
        return set_error(P3M_EUNSUPPORTED, "n * n_sub exceeds the 2^31 receiver-row limit");
    if (!aligned8(pos) || !aligned8(mass) || !aligned8(acc_out))
        return set_error(P3M_EINVAL, "pos, mass and acc_out must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if ((rc = set_device(h))) return rc;
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = rung;
    r.sel_kind = SEL_RUNG;
    r.n_sub = n_sub;
    r.thr = min_rung;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc_out;
    r.stream = (hipStream_t)stream;
    return run(h, r, h->work);
}

int p3m_sr_set_config(p3m_sr_handle h, int subtiles_per_dim, int item_target, int cluster_size,
                      int screen) {
    int rc;
    if (subtiles_per_dim < 0 || subtiles_per_dim > 16)
        return set_error(P3M_EINVAL, "subtiles_per_dim must be in 0..16");
    if (item_target != 0 && (item_target < 64 || item_target > (1 << 20)))
        return set_error(P3M_EINVAL, "item_target must be 0 or in 64..2^20");
    if (cluster_size != 0 && !valid_csize(cluster_size))
        return set_error(P3M_EINVAL, "cluster_size must be 0, 8, 16, 32 or 64");
    if (screen < -1 || screen > 2) return set_error(P3M_EINVAL, "screen must be -1, 0, 1 or 2");
    if (screen == kScreenMutual && cluster_size != 0 && cluster_size < 16)
        return set_error(P3M_EINVAL, "screen 2 needs cluster_size 16, 32 or 64");
    if ((rc = check_handle(h))) return rc;
    h->cfg_ns = subtiles_per_dim;
    h->cfg_target = item_target;
    h->cfg_csize = cluster_size;
    h->cfg_screen = screen;
    return P3M_OK;
}

}  // extern "C"

namespace {

// Measure-and-keep over the candidate layouts for request r (section 2.1.3,
// "Subtiles": try a subdivision, time it, keep it if faster), filed under
// `key`.  The occupancy signature of the inputs is taken from a first call;
// unless level has P3M_TUNE_FORCE, a cached result for this device, key and
// a matching signature is installed without timing anything.
int tune(p3m_sr_context *h, Request &r, const TuneKey &key, int level,
         const std::vector<int> &ns_list, const std::vector<std::pair<int, int>> &layouts,
         const std::vector<int> &targets, const std::vector<int> &targets2, int reps) {
    hipStream_t s = r.stream;
    int rc;
    h->tune_trials = 0;
    h->tune_from_cache = 0;
    // signature of the particle set, from the sort of a first call
    TuneEntry entry;
    entry.device = h->device_id;
    entry.key = key;
    if ((rc = run(h, r, h->work))) return rc;
    if (r.n > 0) {
        const p3m_sr_stats &st = h->stats;
        const Geom g = make_geom(r.box, r.x_s, r.r_cut, st.tiles_per_dim, st.subtiles_per_dim,
                                 0.0);
        if ((rc = ensure(h, h->tune_sig, kSigBins * sizeof(int), s))) return rc;
        int *hist = (int *)h->tune_sig.p;
        P3M_HIP(launch_tile_hist((const int *)h->work.cells.p, g, hist, s));
        P3M_HIP(hipMemcpyAsync(entry.sig, hist, sizeof(entry.sig), hipMemcpyDeviceToHost, s));
        P3M_HIP(hipStreamSynchronize(s));
    }
    // the key under which the fastest layout other than the mutual one is
    // kept, when the mutual one wins
    TuneKey plain_key = key;
    plain_key.kind = plain_kind(key.kind);
    if (!(level & P3M_TUNE_FORCE)) {
        for (const TuneEntry &e : h->cache) {
            if (e.device == h->device_id && e.key == key &&
                sig_distance(e.sig, entry.sig) <= kSigMatch) {
                h->tuned[key] = e.val;
                h->tuned.erase(plain_key);
                for (const TuneEntry &p : h->cache)
                    if (plain_key.kind >= 0 && p.device == h->device_id && p.key == plain_key &&
                        sig_distance(p.sig, entry.sig) <= kSigMatch)
                        h->tuned[plain_key] = p.val;
                h->tune_from_cache = 1;
                return P3M_OK;
            }
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    P3M_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(P3M_EHIP, "hipEventCreate failed");
    }
    struct EventGuard {
        hipEvent_t a, b;
        ~EventGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    float best = 1e30f;
    TuneVal best_v{pick_subtiles(key.nt, r.n, 0), 1024, kDefaultCsize, kDefaultScreen};
    // every candidate's time per call, for the final re-timing of the fastest
    std::vector<std::pair<float, TuneVal>> seen;
    auto time_layout = [&](const TuneVal &v, int nrep, float *per_call) -> int {
        r.force_ns = v.ns;
        r.force_target = v.target;
        r.force_csize = v.csize;
        r.force_screen = v.screen + 1;
        int rc2;
        if ((rc2 = run(h, r, h->work))) return rc2;   // warm-up (also grows the workspace)
        float tot = 0;
        for (int k = 0; k < nrep; ++k) {
            P3M_HIP(hipEventRecord(e0, s));
            if ((rc2 = run(h, r, h->work))) return rc2;
            P3M_HIP(hipEventRecord(e1, s));
            P3M_HIP(hipEventSynchronize(e1));
            float ms = 0;
            P3M_HIP(hipEventElapsedTime(&ms, e0, e1));
            tot += ms;
        }
        *per_call = tot / nrep;
        return P3M_OK;
    };
    auto trial = [&](const TuneVal &v) -> int {
        float ms = 0;
        int rc2;
        if ((rc2 = time_layout(v, reps, &ms))) return rc2;
        ++h->tune_trials;
        seen.push_back({ms, v});
        // a later candidate must be faster by more than the run-to-run noise
        // (about 2 %), so that near-ties do not flip the layout between runs
        if (ms < best * 0.97f) {
            best = ms;
            best_v = v;
        }
        return P3M_OK;
    };
    for (int ns : ns_list) {
        if (pick_subtiles(key.nt, r.n, ns) != ns) continue;
        for (const auto &l : layouts)
            for (int tg : targets)
                if ((rc = trial(TuneVal{ns, tg, l.first, l.second}))) return rc;
    }
    if ((level & 3) >= 2) {
        const TuneVal base = best_v;
        for (int tg : targets2)
            if ((rc = trial(TuneVal{base.ns, tg, base.csize, base.screen}))) return rc;
    }
    // The three fastest candidates are timed again, with twice the calls
    // each, and the fastest of them wins outright: one noisy trial early in
    // the sweep (which later candidates must beat by 3 %) cannot decide.
    std::sort(seen.begin(), seen.end(),
              [](const std::pair<float, TuneVal> &a, const std::pair<float, TuneVal> &b) {
                  return a.first < b.first;
              });
    // re-time the three fastest of the candidates that `keep` accepts; the
    // fastest of them wins outright
    auto retime = [&](bool (*keep)(const TuneVal &), TuneVal *win, float *win_ms) -> int {
        *win_ms = 1e30f;
        int timed = 0;
        for (size_t k = 0; k < seen.size() && timed < 3; ++k) {
            if (!keep(seen[k].second)) continue;
            float ms = 0;
            int rc2;
            if ((rc2 = time_layout(seen[k].second, 2 * reps, &ms))) return rc2;
            ++h->tune_trials;
            ++timed;
            if (ms < *win_ms) {
                *win_ms = ms;
                *win = seen[k].second;
            }
        }
        return P3M_OK;
    };
    if (seen.size() > 1) {
        float final_best = 1e30f;
        if ((rc = retime([](const TuneVal &) { return true; }, &best_v, &final_best))) return rc;
        best = final_best;
    }
    // A mutual winner serves only the calls that can pair once for both
    // partners; the others take the fastest of the remaining layouts.
    bool have_plain = false;
    TuneVal plain_v{};
    float plain_ms = 1e30f;
    if (plain_key.kind >= 0 && best_v.screen == kScreenMutual) {
        if ((rc = retime([](const TuneVal &v) { return v.screen != kScreenMutual; }, &plain_v,
                         &plain_ms)))
            return rc;
        have_plain = plain_ms < 1e30f;
    }
    r.force_ns = r.force_target = r.force_csize = r.force_screen = 0;
    auto file = [&](const TuneKey &k, const TuneVal &v, float ms) {
        h->tuned[k] = v;
        TuneEntry e2 = entry;
        e2.key = k;
        e2.val = v;
        e2.ms = ms;
        bool replaced = false;
        for (TuneEntry &e : h->cache)
            if (e.device == e2.device && e.key == k) {
                e = e2;
                replaced = true;
            }
        if (!replaced) h->cache.push_back(e2);
    };
    file(key, best_v, best);
    if (have_plain) {
        file(plain_key, plain_v, plain_ms);
    } else if (plain_key.kind >= 0) {
        // no longer needed: the winner serves every call
        h->tuned.erase(plain_key);
        h->cache.erase(std::remove_if(h->cache.begin(), h->cache.end(),
                                      [&](const TuneEntry &e) {
                                          return e.device == h->device_id && e.key == plain_key;
                                      }),
                       h->cache.end());
    }
    save_cache(h);
    return P3M_OK;
}

}  // namespace

extern "C" {

int p3m_sr_autotune(p3m_sr_handle h, const double *pos, const double *mass, const uint8_t *active,
                    int64_t n, double box, double x_s, double r_cut, int precision, int level,
                    double *acc_scratch, void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    const bool adjoint = (level & P3M_TUNE_ADJOINT) != 0;
    const int base_level = level & ~(P3M_TUNE_ADJOINT | P3M_TUNE_FORCE);
    if (base_level < 1 || base_level > 2)
        return set_error(P3M_EINVAL,
                         "level must be 1 or 2, optionally | P3M_TUNE_ADJOINT | P3M_TUNE_FORCE");
    if (n > 0 && (!pos || !acc_scratch))
        return set_error(P3M_EINVAL, "pos and acc_scratch are required");
    if (!aligned8(pos) || !aligned8(mass) || !aligned8(acc_scratch))
        return set_error(P3M_EINVAL, "pos, mass and acc_scratch must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)stream;
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = active;
    r.sel_kind = active ? SEL_MASK : SEL_ALL;
    r.n_sub = 1;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc_scratch;
    r.stream = s;
    if (adjoint) {
        // the adjoint's trials take unit weights on every receiver as grad_acc
        if ((rc = ensure(h, h->tune_w, ((size_t)n + 1) * 3 * sizeof(double), s))) return rc;
        P3M_HIP(launch_fill_f64((double *)h->tune_w.p, 1.0, (size_t)n * 3, s));
        r.backward = true;
        r.grad_acc = (const double *)h->tune_w.p;
    }
    const int nt = tiles_per_dim(box, r_cut);
    // level 1: subtiles x layout (cluster size, screening) x two item sizes;
    // level 2 also sweeps the item size around the level-1 winner
    std::vector<std::pair<int, int>> layouts = {{64, 0}, {64, 1}, {32, 1}, {16, 1}, {8, 1},
                                                {16, 0}, {8, 0}};
    // all-active forward calls (softened or not; FP32 ones with the
    // polynomial shape) and adjoints without softening can evaluate each pair
    // once for both partners
    const bool fp32_t = precision == P3M_FP32;
    if (adjoint ? h->eps == 0.0 : (!active && (!fp32_t || h->cfg_shape == SHAPE_POLY)))
        for (int c : {32, 64, 16}) layouts.push_back({c, kScreenMutual});
    const TuneKey key{n, nt, precision, adjoint ? TUNE_ADJOINT : TUNE_FORWARD, 1};
    rc = tune(h, r, key, level, {1, 2, 3, 4}, layouts, {1024, 4096},
              {256, 512, 2048, 8192, 16384}, 3);
    if (rc) return rc;
    // until it is tuned on its own, the adjoint takes the forward's winner
    // (and the forward's layout for the calls the winner cannot serve)
    if (!adjoint) {
        const TuneKey adj{n, nt, precision, TUNE_ADJOINT, 1};
        const TuneKey fwd_plain{n, nt, precision, TUNE_FORWARD_PLAIN, 1};
        const TuneKey adj_plain{n, nt, precision, TUNE_ADJOINT_PLAIN, 1};
        if (!h->tuned.count(adj)) {
            h->tuned[adj] = h->tuned[key];
            auto p = h->tuned.find(fwd_plain);
            if (p != h->tuned.end()) h->tuned[adj_plain] = p->second;
        }
    }
    return P3M_OK;
}

int p3m_sr_autotune_batched(p3m_sr_handle h, const double *pos, const double *mass,
                            const uint8_t *rung, int64_t n, int n_sub, const uint8_t *min_rung,
                            double box, double x_s, double r_cut, int precision, int level,
                            double *acc_scratch, void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    const int base_level = level & ~P3M_TUNE_FORCE;
    if (base_level < 1 || base_level > 2)
        return set_error(P3M_EINVAL, "level must be 1 or 2, optionally | P3M_TUNE_FORCE");
    if (n_sub < 1 || n_sub > 64) return set_error(P3M_EINVAL, "n_sub must be in 1..64");
    if (!min_rung) return set_error(P3M_EINVAL, "min_rung (host array) is required");
    if (n > 0 && (!pos || !rung || !acc_scratch))
        return set_error(P3M_EINVAL, "pos, rung and acc_scratch are required");
    if ((double)n * n_sub > 2.0e9)
        return set_error(P3M_EUNSUPPORTED, "n * n_sub exceeds the 2^31 receiver-row limit");
    if (!aligned8(pos) || !aligned8(mass) || !aligned8(acc_scratch))
        return set_error(P3M_EINVAL, "pos, mass and acc_scratch must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if ((rc = set_device(h))) return rc;
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = rung;
    r.sel_kind = SEL_RUNG;
    r.n_sub = n_sub;
    r.thr = min_rung;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc_scratch;
    r.stream = (hipStream_t)stream;
    const int nt = tiles_per_dim(box, r_cut);
    // a batched call is long (every subset's pairs): fewer candidates (the
    // screened layouts), each timed once after its warm-up call
    const std::vector<std::pair<int, int>> layouts = {{32, 1}, {16, 1}, {64, 1}};
    return tune(h, r, TuneKey{n, nt, precision, TUNE_BATCHED, n_sub}, level, {1, 2}, layouts,
                {4096}, {1024, 16384}, 1);
}

int p3m_sr_set_tune_cache(p3m_sr_handle h, const char *path) {
    int rc;
    if ((rc = check_handle(h))) return rc;
    h->cache_path = path ? std::string(path) : default_cache_path();
    load_cache(h);
    return P3M_OK;
}

int p3m_sr_tune_cache_check(const char *path, int *entries, int *lines) {
    if (!path) return set_error(P3M_EINVAL, "NULL path");
    std::vector<TuneEntry> v;
    int nl = 0;
    if (!read_cache_file(path, v, &nl))
        return set_error(P3M_EINVAL, "cannot open the cache file %.200s", path);
    if (entries) *entries = (int)v.size();
    if (lines) *lines = nl;
    return P3M_OK;
}

int p3m_sr_tune_status(p3m_sr_handle h, int *trials_timed, int *from_cache) {
    int rc;
    if ((rc = check_handle(h))) return rc;
    if (trials_timed) *trials_timed = h->tune_trials;
    if (from_cache) *from_cache = h->tune_from_cache;
    return P3M_OK;
}

int p3m_sr_set_shape(p3m_sr_handle h, int kind, int table_size) {
    int rc;
    if (kind != P3M_SHAPE_POLY && kind != P3M_SHAPE_TAB_NGP && kind != P3M_SHAPE_TAB_LINEAR)
        return set_error(P3M_EINVAL, "unknown shape kind %d", kind);
    const int max_n = kind == P3M_SHAPE_TAB_LINEAR ? kTabFloats / 2 : kTabFloats;
    if (table_size == 0) table_size = kind == P3M_SHAPE_POLY ? 0 : max_n;
    if (kind != P3M_SHAPE_POLY &&
        (table_size < 64 || table_size > max_n || (table_size & (table_size - 1)) != 0))
        return set_error(P3M_EINVAL, "table_size must be a power of two in [64, %d]", max_n);
    if ((rc = check_handle(h))) return rc;
    h->cfg_shape = kind;
    h->cfg_tab_n = kind == P3M_SHAPE_POLY ? 0 : table_size;
    return P3M_OK;
}

int p3m_sr_set_softening(p3m_sr_handle h, double eps) {
    int rc;
    if (!(eps >= 0.0) || !std::isfinite(eps))
        return set_error(P3M_EINVAL, "eps must be finite and >= 0");
    if ((rc = check_handle(h))) return rc;
    h->eps = eps;
    return P3M_OK;
}

int p3m_sr_set_deterministic(p3m_sr_handle h, int enable) {
    int rc;
    if (enable != 0 && enable != 1) return set_error(P3M_EINVAL, "enable must be 0 or 1");
    if ((rc = check_handle(h))) return rc;
    h->deterministic = enable != 0;
    return P3M_OK;
}

int p3m_sr_set_debug_limits(p3m_sr_handle h, int64_t max_workspace_bytes, int fail_after) {
    int rc;
    if (max_workspace_bytes < 0) return set_error(P3M_EINVAL, "max_workspace_bytes must be >= 0");
    if (fail_after < -1) return set_error(P3M_EINVAL, "fail_after must be >= -1");
    if ((rc = check_handle(h))) return rc;
    h->dbg_max_bytes = (size_t)max_workspace_bytes;
    h->dbg_fail_after = fail_after;
    return P3M_OK;
}

int p3m_sr_set_timing(p3m_sr_handle h, int enable) {
    int rc;
    if ((rc = check_handle(h))) return rc;
    h->timing = enable != 0;
    return P3M_OK;
}

int p3m_sr_get_stats(p3m_sr_handle h, p3m_sr_stats *out) {
    int rc;
    if ((rc = check_handle(h))) return rc;
    if (!out) return set_error(P3M_EINVAL, "NULL stats pointer");
    if ((rc = set_device(h))) return rc;
    p3m_sr_stats st = h->stats;
    if (st.n > 0 && st.items < 0) {
        // the totals of the latest run of the call (k_totals writes them to
        // pinned memory; a graph replay of the call writes them again)
        P3M_HIP(hipStreamSynchronize(h->last_stream));
        st.receivers = h->host_tot[0];
        st.clusters = h->host_tot[1];
        st.items = h->host_tot[2];
    }
    if (h->last_counters && st.n > 0) {
        Counters cp[kCounterCopies * kCounterStride];
        P3M_HIP(hipStreamSynchronize(h->last_stream));
        P3M_HIP(hipMemcpy(cp, h->last_counters, sizeof(cp), hipMemcpyDeviceToHost));
        Counters c{};
        for (int k = 0; k < kCounterCopies; ++k) {
            const Counters &e = cp[k * kCounterStride];
            c.interactions += e.interactions;
            c.candidates += e.candidates;
            c.steps += e.steps;
            c.screened += e.screened;
            c.rare += e.rare;
            c.scan_stall += e.scan_stall;
        }
        st.interactions = (int64_t)c.interactions;
        st.candidates = (int64_t)c.candidates;
        st.steps = (int64_t)c.steps;
        st.screened = (int64_t)c.screened;
        st.fp64_steps = (int64_t)c.rare;
        if (c.scan_stall)
            return set_error(P3M_EHIP, "a scan of the last call waited past its poll limit "
                                       "(its result is not valid)");
    }
    if (h->timed_last) {
        float a = 0, b = 0, t = 0;
        P3M_HIP(hipEventSynchronize(h->ev[3]));
        P3M_HIP(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
        P3M_HIP(hipEventElapsedTime(&b, h->ev[1], h->ev[2]));
        P3M_HIP(hipEventElapsedTime(&t, h->ev[0], h->ev[3]));
        P3M_HIP(hipEventElapsedTime(&st.ms_sort, h->ev[0], h->ev[4]));
        if (h->sort_b) {
            float sb = 0;
            P3M_HIP(hipEventSynchronize(h->ev[5]));
            P3M_HIP(hipEventElapsedTime(&sb, h->ev[0], h->ev[5]));
            st.ms_sort = std::max(st.ms_sort, sb);
        }
        st.ms_build = a;
        st.ms_pairs = b;
        st.ms_total = t;
    }
    *out = st;
    return P3M_OK;
}

int p3m_lr_force(p3m_sr_handle h, const double *pos, const double *mass, const uint8_t *active,
                 int64_t n, double box, int n_grid, double x_s, double *acc_out, void *stream) {
    int rc;
    if (n < 0) return set_error(P3M_EINVAL, "n must be >= 0");
    if (!(box > 0.0) || !std::isfinite(box)) return set_error(P3M_EINVAL, "box must be > 0");
    if (!(x_s > 0.0) || !std::isfinite(x_s)) return set_error(P3M_EINVAL, "x_s must be > 0");
    if (n_grid < 16 || n_grid > 1024 || (n_grid & (n_grid - 1)) != 0)
        return set_error(P3M_EINVAL, "n_grid must be a power of two in [16, 1024], got %d",
                         n_grid);
    if (n > 0 && (!pos || !acc_out)) return set_error(P3M_EINVAL, "pos and acc_out are required");
    if (!aligned8(pos) || !aligned8(acc_out) || !aligned8(mass))
        return set_error(P3M_EINVAL, "pos, mass and acc_out must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if (n > (int64_t)0x7ffffff0)
        return set_error(P3M_EUNSUPPORTED, "more than 2^31 - 16 particles");
    if ((rc = set_device(h))) return rc;
    return lr_run(h, pos, mass, active, (int)n, box, n_grid, x_s, acc_out,
                  (hipStream_t)stream);
}

int p3m_lr_get_stats(p3m_sr_handle h, p3m_lr_stats *out) {
    int rc;
    if ((rc = check_handle(h))) return rc;
    if (!out) return set_error(P3M_EINVAL, "NULL stats pointer");
    if ((rc = set_device(h))) return rc;
    p3m_lr_stats st = h->lr_stats;
    float *ms[9] = {nullptr,          &st.ms_sort,       &st.ms_deposit,
                    &st.ms_fft_x_fwd, &st.ms_fft_y_fwd,  &st.ms_fft_z_conv,
                    &st.ms_fft_y_inv, &st.ms_fft_x_inv,  &st.ms_readout};
    for (int k = 1; k < 9; ++k) *ms[k] = -1.0f;
    st.ms_total = -1.0f;
    if (h->lr_timed) {
        P3M_HIP(hipEventSynchronize(h->lr_ev[8]));
        for (int k = 1; k < 9; ++k)
            P3M_HIP(hipEventElapsedTime(ms[k], h->lr_ev[k - 1], h->lr_ev[k]));
        P3M_HIP(hipEventElapsedTime(&st.ms_total, h->lr_ev[0], h->lr_ev[8]));
    } else if (h->lr_stream || st.n > 0) {
        P3M_HIP(hipStreamSynchronize(h->lr_stream));
    }
    *out = st;
    return P3M_OK;
}

int p3m_kdk_step(p3m_sr_handle h, double *pos, double *vel, const double *mass, uint8_t *rung,
                 int64_t n, double box, double x_s, double r_cut, int n_grid, double dt,
                 int n_steps, double eta, double eps, int max_rung, int flags, int precision,
                 void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    if (n_grid != 0 && (n_grid < 16 || n_grid > 1024 || (n_grid & (n_grid - 1)) != 0))
        return set_error(P3M_EINVAL, "n_grid must be 0 or a power of two in [16, 1024], got %d",
                         n_grid);
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(P3M_EINVAL, "dt must be > 0");
    if (n_steps < 1 || n_steps > 64) return set_error(P3M_EINVAL, "n_steps must be in [1, 64]");
    if (max_rung < 0 || max_rung > 7) return set_error(P3M_EINVAL, "max_rung must be in [0, 7]");
    if (flags & ~P3M_KDK_FIXED_RUNGS) return set_error(P3M_EINVAL, "unknown flags 0x%x", flags);
    const bool fixed = (flags & P3M_KDK_FIXED_RUNGS) != 0;
    if (!(eps >= 0.0) || !std::isfinite(eps)) return set_error(P3M_EINVAL, "eps must be >= 0");
    if (!fixed && !(eps > 0.0 && eta > 0.0 && std::isfinite(eta)))
        return set_error(P3M_EINVAL, "eq. rung needs eta > 0 and eps > 0 (or fixed rungs)");
    if (n > 0 && (!pos || !vel || !rung))
        return set_error(P3M_EINVAL, "pos, vel and rung are required");
    if (!aligned8(pos) || !aligned8(vel) || !aligned8(mass))
        return set_error(P3M_EINVAL, "pos, vel and mass must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if (n > (int64_t)0x7ffffff0)
        return set_error(P3M_EUNSUPPORTED, "more than 2^31 - 16 particles");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int np = (int)n;
    const size_t np1 = (size_t)np + 1;
    if ((rc = ensure(h, h->kdk_acc, np1 * 3 * sizeof(double), s))) return rc;
    if (n_grid && (rc = ensure(h, h->kdk_lr, np1 * 3 * sizeof(double), s))) return rc;
    if ((rc = ensure(h, h->kdk_tq, np1 * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->kdk_tnext, np1 * sizeof(int), s))) return rc;
    if ((rc = ensure(h, h->kdk_due, np1, s))) return rc;
    if ((rc = ensure(h, h->kdk_scal, 8 * sizeof(int), s))) return rc;
    double *acc = (double *)h->kdk_acc.p, *acc_lr = (double *)h->kdk_lr.p;
    int *t_q = (int *)h->kdk_tq.p, *t_next = (int *)h->kdk_tnext.p;
    int *scal = (int *)h->kdk_scal.p;   // [0] highest rung, [1] due count, [2..3] pairs
    unsigned long long *pairs = (unsigned long long *)(scal + 2);
    uint8_t *due = (uint8_t *)h->kdk_due.p;

    // the call's softening is eps for both the forces and eq. rung
    struct EpsGuard {
        p3m_sr_context *h;
        double saved;
        ~EpsGuard() { h->eps = saved; }
    } guard{h, h->eps};
    h->eps = eps;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->timing) {
        P3M_HIP(hipEventCreate(&e0));
        P3M_HIP(hipEventCreate(&e1));
        P3M_HIP(hipEventRecord(e0, s));
    }

    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = nullptr;
    r.sel_kind = SEL_ALL;
    r.n_sub = 1;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc;
    r.stream = s;
    int sr_calls = 0, lr_calls = 0;
    // short-range accelerations at the synchronised start: they set the rungs
    // (eq. rung, no momentum update) and drive the half kicks
    P3M_HIP(launch_fill_i32(scal, 0, 8, s));
    if ((rc = run(h, r, h->work))) return rc;
    ++sr_calls;
    if (np > 0) P3M_HIP(launch_kdk_accum(h->last_counters, pairs, s));
    KdkArgs k{};
    k.dt = dt;
    k.two_eta_eps = 2.0 * eta * eps;
    k.max_rung = max_rung;
    k.fixed = fixed ? 1 : 0;
    P3M_HIP(launch_kdk_assign(acc, np, k, rung, scal, s));
    int L = 0;
    P3M_HIP(hipMemcpyAsync(&L, scal, sizeof(int), hipMemcpyDeviceToHost, s));
    P3M_HIP(hipStreamSynchronize(s));
    if (L > max_rung)
        return set_error(P3M_EINVAL, "input rung %d exceeds max_rung %d", L, max_rung);
    k.L = L;
    const double tau = dt / (double)(1 << L);
    k.half_tau = 0.5 * tau;
    k.period = n_steps * (1 << (L + 1));
    const int span0 = 1 << (L + 1);
    P3M_HIP(launch_kdk_first(vel, acc, np, k, rung, t_q, t_next, s));
    int t_lr = 0;
    if (n_grid) {
        if ((rc = lr_run(h, pos, mass, nullptr, np, box, n_grid, x_s, acc_lr, s))) return rc;
        ++lr_calls;
        const int target = span0 / 2;
        P3M_HIP(launch_axpy3(vel, acc_lr, np, (double)(target - t_lr) * k.half_tau, s));
        t_lr = target;
    }
    for (int t = 2; t <= k.period; t += 2) {
        P3M_HIP(launch_kdk_drift(pos, vel, np, tau, box, s));
        P3M_HIP(launch_fill_i32(scal + 1, 0, 1, s));
        P3M_HIP(launch_kdk_due(t_next, np, t, due, scal + 1, s));
        int n_due = 0;
        P3M_HIP(hipMemcpyAsync(&n_due, scal + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        P3M_HIP(hipStreamSynchronize(s));
        if (n_due > 0) {
            r.sel = due;
            r.sel_kind = SEL_MASK;
            if ((rc = run(h, r, h->work))) return rc;
            ++sr_calls;
            P3M_HIP(launch_kdk_accum(h->last_counters, pairs, s));
            P3M_HIP(launch_kdk_kick(vel, acc, due, np, t, k, rung, t_q, t_next, s));
        }
        if (n_grid && t % span0 == 0) {
            if ((rc = lr_run(h, pos, mass, nullptr, np, box, n_grid, x_s, acc_lr, s))) return rc;
            ++lr_calls;
            const int target = t == k.period ? k.period : t + span0 / 2;
            P3M_HIP(launch_axpy3(vel, acc_lr, np, (double)(target - t_lr) * k.half_tau, s));
            t_lr = target;
        }
    }
    h->kdk_stats = p3m_kdk_stats{};
    h->kdk_stats.n = n;
    h->kdk_stats.highest_rung = L;
    h->kdk_stats.substeps = k.period / 2;
    h->kdk_stats.sr_calls = sr_calls;
    h->kdk_stats.lr_calls = lr_calls;
    h->kdk_stats.ms_total = -1.0f;
    unsigned long long total = 0;
    P3M_HIP(hipMemcpyAsync(&total, pairs, sizeof(total), hipMemcpyDeviceToHost, s));
    P3M_HIP(hipStreamSynchronize(s));
    h->kdk_stats.interactions = (int64_t)total;
    if (e0) {
        P3M_HIP(hipEventRecord(e1, s));
        P3M_HIP(hipEventSynchronize(e1));
        P3M_HIP(hipEventElapsedTime(&h->kdk_stats.ms_total, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return P3M_OK;
}

int p3m_force(p3m_sr_handle h, const double *pos, const double *mass, const uint8_t *active,
              int64_t n, double box, double x_s, double r_cut, int n_grid, int precision,
              double *acc_out, void *stream) {
    int rc;
    if ((rc = check_geometry(n, box, x_s, r_cut))) return rc;
    if (precision != P3M_FP32 && precision != P3M_FP64)
        return set_error(P3M_EINVAL, "precision must be P3M_FP64 or P3M_FP32");
    if (n_grid < 16 || n_grid > 1024 || (n_grid & (n_grid - 1)) != 0)
        return set_error(P3M_EINVAL, "n_grid must be a power of two in [16, 1024], got %d",
                         n_grid);
    if (n > 0 && (!pos || !acc_out)) return set_error(P3M_EINVAL, "pos and acc_out are required");
    if (!aligned8(pos) || !aligned8(acc_out) || !aligned8(mass))
        return set_error(P3M_EINVAL, "pos, mass and acc_out must be 8-byte aligned");
    if ((rc = check_handle(h))) return rc;
    if (n > (int64_t)0x7ffffff0)
        return set_error(P3M_EUNSUPPORTED, "more than 2^31 - 16 particles");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int np = (int)n;
    if (!h->aux) {
        P3M_HIP(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
        P3M_HIP(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
        P3M_HIP(hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming));
    }
    if ((rc = ensure(h, h->p3m_lr, ((size_t)np + 1) * 3 * sizeof(double), s))) return rc;
    // the long range waits for the caller's earlier work, then runs on the
    // auxiliary stream while the short range runs on the caller's
    P3M_HIP(hipEventRecord(h->fork_ev, s));
    P3M_HIP(hipStreamWaitEvent(h->aux, h->fork_ev, 0));
    rc = lr_run(h, pos, mass, active, np, box, n_grid, x_s, (double *)h->p3m_lr.p, h->aux);
    P3M_HIP(hipEventRecord(h->join_ev, h->aux));
    if (rc) {
        // whatever the long range queued still finishes before later work on `stream`
        P3M_HIP(hipStreamWaitEvent(s, h->join_ev, 0));
        return rc;
    }
    Request r{};
    r.pos = pos;
    r.mass = mass;
    r.sel = active;
    r.sel_kind = active ? SEL_MASK : SEL_ALL;
    r.n_sub = 1;
    r.n = n;
    r.box = box;
    r.x_s = x_s;
    r.r_cut = r_cut;
    r.precision = precision;
    r.out = acc_out;
    r.stream = s;
    rc = run(h, r, h->work);
    // join before returning, also when the short range failed
    P3M_HIP(hipStreamWaitEvent(s, h->join_ev, 0));
    if (rc) return rc;
    P3M_HIP(launch_axpy3(acc_out, (const double *)h->p3m_lr.p, np, 1.0, s));
    h->last_stream = s;
    return P3M_OK;
}

int p3m_kdk_get_stats(p3m_sr_handle h, p3m_kdk_stats *out) {
    int rc;
    if ((rc = check_handle(h))) return rc;
    if (!out) return set_error(P3M_EINVAL, "NULL stats pointer");
    *out = h->kdk_stats;
    return P3M_OK;
}

}  // extern "C"
