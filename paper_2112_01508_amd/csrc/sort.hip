// Tile/subtile counting sort, receiver compaction and work-item planning.
//
// Section 2.1.3 ("Tiles", "Subtiles", "Other optimisations"): particles are
// sorted in O(N) into tiles of side >= r_cut, each split into ns^3
// subtiles, and stored in tile -> subtile -> particle order.  On the GPU the
// sort is a counting sort over the fine cells (histogram with atomics ->
// exclusive scan -> scatter).  Receivers (the particles on active rungs,
// section 2.2.2) are compacted per tile and grouped into clusters of at most
// one wavefront; each cluster is then split into work items over its 27
// neighbour tiles so that one persistent launch can balance the very uneven
// work of clustered particle sets.
#include "p3msr_internal.hpp"

#include <algorithm>
#include <climits>

namespace p3m {

namespace {

__global__ void k_fill_i32(int *p, int v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    if (((uintptr_t)p & 15) == 0) {
        // 16-byte stores for the bulk, then the tail
        int4 *p4 = reinterpret_cast<int4 *>(p);
        const size_t n4 = n / 4;
        const int4 v4 = make_int4(v, v, v, v);
        for (size_t j = i; j < n4; j += stride) p4[j] = v4;
        for (size_t j = 4 * n4 + i; j < n; j += stride) p[j] = v;
        return;
    }
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Position wrapped into [0, box).
__device__ inline double wrap_coord(double x, const Geom &g) {
    double w = x - g.box * floor(x * g.inv_box);
    if (!(w < g.box)) w = 0.0;   // rounding up to box, or NaN
    if (w < 0.0) w = 0.0;
    return w;
}

__device__ inline int cell_of(double w, const Geom &g) {
    int c = (int)(w * g.inv_cell);
    return c < 0 ? 0 : (c >= g.nc ? g.nc - 1 : c);
}

__device__ inline int key_of(int cx, int cy, int cz, const Geom &g) {
    int tx = cx / g.ns, ty = cy / g.ns, tz = cz / g.ns;
    int sx = cx - tx * g.ns, sy = cy - ty * g.ns, sz = cz - tz * g.ns;
    int tile = (tx * g.nt + ty) * g.nt + tz;
    return tile * g.ns3 + (sx * g.ns + sy) * g.ns + sz;
}

// Cell key and rank inside the cell, with one global atomic per distinct
// cell of a block of kKeysThreads x PPT particles: the block's keys are
// counted in an LDS hash table first (a dense halo cell's particles, which
// share blocks, would otherwise hit one counter from every wave that holds
// any of them, and those atomics serialise on its address).  The global
// atomics bound the kernel, so larger blocks (more particles sharing a cell)
// pay off.
constexpr int kKeysThreads = 1024;

template <int PPT>
__global__ __launch_bounds__(kKeysThreads) void k_keys(const double *__restrict__ pos, int n,
                                                       Geom g, int *__restrict__ key,
                                                       int *__restrict__ rank,
                                                       int *__restrict__ cell_count) {
    constexpr int kSlots = 2 * kKeysThreads * PPT;   // open addressing, at most half full
    constexpr int kShift = 32 - __builtin_ctz(kSlots);
    __shared__ int skey[kSlots];
    __shared__ int scnt[kSlots];
    for (int t = threadIdx.x; t < kSlots; t += blockDim.x) {
        skey[t] = -1;
        scnt[t] = 0;
    }
    __syncthreads();
    int slot[PPT], local[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const long long i = ((long long)blockIdx.x * PPT + p) * kKeysThreads + threadIdx.x;
        slot[p] = -1;
        local[p] = 0;
        if (i < n) {
            const double wx = wrap_coord(pos[3 * (size_t)i], g);
            const double wy = wrap_coord(pos[3 * (size_t)i + 1], g);
            const double wz = wrap_coord(pos[3 * (size_t)i + 2], g);
            const int k = key_of(cell_of(wx, g), cell_of(wy, g), cell_of(wz, g), g);
            key[i] = k;
            // k >= 0 and the table never fills, so the probe ends
            int sl = (int)(((unsigned)k * 2654435761u) >> kShift);
            for (;;) {
                const int old = atomicCAS(&skey[sl], -1, k);
                if (old == -1 || old == k) break;
                sl = (sl + 1) & (kSlots - 1);
            }
            slot[p] = sl;
            local[p] = atomicAdd(&scnt[sl], 1);
        }
    }
    __syncthreads();
    // one global atomic per occupied slot; its base replaces the count
    for (int t = threadIdx.x; t < kSlots; t += blockDim.x) {
        const int kk = skey[t];
        if (kk >= 0) scnt[t] = atomicAdd(&cell_count[kk], scnt[t]);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const long long i = ((long long)blockIdx.x * PPT + p) * kKeysThreads + threadIdx.x;
        if (slot[p] >= 0) rank[i] = scnt[slot[p]] + local[p];
    }
}
// ---- exclusive scan (reduce / top / down-sweep) -----------------------------

__device__ inline int block_exclusive_scan(int v, int *lds, int *total) {
    // wave-level inclusive scan with shuffles, then across the block's waves
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    int x = v;
    for (int off = 1; off < kWave; off <<= 1) {
        int y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) lds[wave] = x;
    __syncthreads();
    const int nw = blockDim.x / kWave;
    int base = 0, all = 0;
    for (int w = 0; w < nw; ++w) {
        int s = lds[w];
        if (w < wave) base += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return base + x - v;
}

// Tiles of kScanTile values; a block's threads load them striped (value
// k * kScanBlock + t), so every wave load is coalesced.
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int *__restrict__ in, size_t n,
                                                            int *__restrict__ bsum) {
    __shared__ int lds[kScanBlock / kWave];
    const size_t base = (size_t)blockIdx.x * kScanTile + threadIdx.x;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        const size_t i = base + (size_t)k * kScanBlock;
        if (i < n) s += in[i];
    }
    int total;
    block_exclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(int *__restrict__ bsum, int nb,
                                                   int *__restrict__ out_total) {
    __shared__ int lds[1024 / kWave];
    int carry = 0;
    for (int base = 0; base < nb; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        int total;
        int ex = block_exclusive_scan(v, lds, &total);
        if (i < nb) bsum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        bsum[nb] = carry;
        *out_total = carry;
    }
}

// Down-sweep: the tile is loaded striped into LDS, each thread scans its
// kScanPerThread consecutive values there (a pad word per 16 keeps the
// per-thread reads free of bank conflicts), and the result is stored striped.
// in and out may be the same array.
__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 4); }

__global__ __launch_bounds__(kScanBlock) void k_scan_down(const int *in, int *out, size_t n,
                                                          const int *__restrict__ bsum) {
    __shared__ int lds[kScanBlock / kWave];
    __shared__ int tile[kScanTile + kScanTile / 16];
    const size_t base = (size_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        const int e = k * kScanBlock + threadIdx.x;
        const size_t i = base + e;
        tile[scan_pad(e)] = i < n ? in[i] : 0;
    }
    __syncthreads();
    const int first = threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = tile[scan_pad(first + k)];
        s += v[k];
    }
    int total;
    int run = block_exclusive_scan(s, lds, &total) + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        tile[scan_pad(first + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        const int e = k * kScanBlock + threadIdx.x;
        const size_t i = base + e;
        if (i < n) out[i] = tile[scan_pad(e)];
    }
}

// Single-pass exclusive scan (decoupled look-back).  Each block takes the
// next tile number from a counter, so every tile before it belongs to a
// block that is already running; it scans its tile, publishes the tile's
// sum at once (nothing delays that), then its first wave reads the status of
// the 64 tiles before it together, adding their sums back to the nearest
// published inclusive prefix (another window of 64 if there is none), and
// publishes its own.  status[t] (zeroed before the launch): 0 nothing yet,
// 1 << 32 | sum, or 2 << 32 | inclusive prefix.  A wait longer than
// kScan1Spins polls (which a running predecessor cannot cause) ends the wait
// anyway and raises *stall.  out[n] = the total; in may equal out.
constexpr unsigned long long kScanSum = 1ull << 32, kScanPrefix = 2ull << 32;
constexpr int kScan1Spins = 1 << 20;
constexpr int kScan1MaxTiles = 64;   // larger scans take the three-kernel path

__global__ __launch_bounds__(kScanBlock) void k_scan_1pass(const int *in, int *out, size_t n,
                                                           unsigned long long *status, int *ctr,
                                                           unsigned long long *stall) {
    __shared__ int lds[kScanBlock / kWave];
    __shared__ int tile[kScanTile + kScanTile / 16];
    __shared__ int s_tile, s_excl;
    if (threadIdx.x == 0) s_tile = atomicAdd(ctr, 1);
    __syncthreads();
    const int t = s_tile;
    const size_t base = (size_t)t * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        const int e = k * kScanBlock + threadIdx.x;
        const size_t i = base + e;
        tile[scan_pad(e)] = i < n ? in[i] : 0;
    }
    __syncthreads();
    const int first = threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = tile[scan_pad(first + k)];
        sum += v[k];
    }
    int total;
    int run = block_exclusive_scan(sum, lds, &total);
    if (threadIdx.x < kWave) {
        // the first wave: publish the tile's sum, then look back over the
        // 64 tiles before the window's top at once; tiles before 0 count as
        // a prefix of 0, so every window that reaches them ends the walk
        const int lane = threadIdx.x;
        if (lane == 0)
            __hip_atomic_store(&status[t], (t == 0 ? kScanPrefix : kScanSum) | (unsigned)total,
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int excl = 0;
        for (int top = t - 1; top >= 0; top -= kWave) {
            const int p = top - lane;
            int spins = 0;
            int near = kWave;   // lowest lane (nearest tile) holding a prefix
            unsigned long long st = 0;
            for (;;) {
                st = p >= 0 ? __hip_atomic_load(&status[p], __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                            : kScanPrefix;
                const unsigned long long pm = __builtin_amdgcn_ballot_w64((st >> 32) == 2);
                const unsigned long long em = __builtin_amdgcn_ballot_w64((st >> 32) == 0);
                near = pm ? __builtin_ctzll(pm) : kWave;
                const unsigned long long need =
                    near >= kWave - 1 ? ~0ull : ((2ull << near) - 1ull);
                if ((em & need) == 0) break;
                if (++spins >= kScan1Spins) {
                    if (lane == 0) atomicAdd(stall, 1ull);
                    near = -1;   // give up: the result is flagged as invalid
                    break;
                }
            }
            if (near < 0) break;
            int add = lane <= near ? (int)(unsigned)(st & 0xffffffffull) : 0;
            for (int off = kWave / 2; off > 0; off >>= 1) add += __shfl_xor(add, off, kWave);
            excl += add;
            if (near < kWave) break;
        }
        if (lane == 0) {
            if (t > 0)
                __hip_atomic_store(&status[t], kScanPrefix | (unsigned)(excl + total),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            s_excl = excl;
            if (base + kScanTile >= n) out[n] = excl + total;   // the last tile
        }
    }
    __syncthreads();
    run += s_excl;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        tile[scan_pad(first + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        const int e = k * kScanBlock + threadIdx.x;
        const size_t i = base + e;
        if (i < n) out[i] = tile[scan_pad(e)];
    }
}

// ---- scatter into tile -> subtile order --------------------------------------

// Particles of subtiles with at most keep_max particles keep their scattered
// order, so they go straight to the final arrays (sp_f, perm_f, sel_f); the
// others go to the staging arrays that the fine-order pass reorders from.
__global__ void k_scatter(const double *__restrict__ pos, const double *__restrict__ mass,
                          const uint8_t *__restrict__ sel, int n, Geom g,
                          const int *__restrict__ key, const int *__restrict__ rank,
                          const int *__restrict__ cell_start, int fp32, int keep_max,
                          double4 *__restrict__ sp_s, int *__restrict__ perm_s,
                          uint8_t *__restrict__ sel_st, double4 *__restrict__ sp_f,
                          int *__restrict__ perm_f, uint8_t *__restrict__ sel_f) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = key[i];
    const int c0 = cell_start[k];
    int dst = c0 + rank[i];
    const bool direct = cell_start[k + 1] - c0 <= keep_max;
    double4 *__restrict__ sp = direct ? sp_f : sp_s;
    int *__restrict__ perm = direct ? perm_f : perm_s;
    uint8_t *__restrict__ sel_s = direct ? sel_f : sel_st;
    double4 v;
    v.x = wrap_coord(pos[3 * (size_t)i], g);
    v.y = wrap_coord(pos[3 * (size_t)i + 1], g);
    v.z = wrap_coord(pos[3 * (size_t)i + 2], g);
    double mu = mass ? mass[i] : 1.0;
    if (fp32) {
        float mf = (float)mu;
        v.w = __longlong_as_double((long long)(unsigned int)__float_as_uint(mf));
    } else {
        v.w = mu;
    }
    sp[dst] = v;
    perm[dst] = i;
    if (sel) sel_s[dst] = sel[i];   // no selector: every particle takes part
}

// ---- fine order inside subtiles -------------------------------------------------

// Morton index of the particle's 8x8x8 sub-cell inside its subtile.
__device__ inline int fine_key(const double4 &p, const Geom &g) {
    int f[3];
    const double w[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = w[d] * g.inv_cell;
        int c = (int)u;
        c = c < 0 ? 0 : (c >= g.nc ? g.nc - 1 : c);
        int q = (int)((u - c) * kFineSide);
        f[d] = q < 0 ? 0 : (q >= kFineSide ? kFineSide - 1 : q);
    }
    int k = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b)
        k |= (((f[0] >> b) & 1) << (3 * b + 2)) | (((f[1] >> b) & 1) << (3 * b + 1)) |
             (((f[2] >> b) & 1) << (3 * b));
    return k;
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Fine order, medium subtiles: one wave per tile, kFineWaves tiles per
// block.  Inside every subtile holding more than keep_max and at most
// kFineBig particles the particles are reordered by fine_key (a counting sort
// over kFineBins bins in LDS); smaller subtiles are already in place (the
// scatter wrote them to sp2/perm2/sel2); larger ones are k_fine_order_big's,
// which can run at the same time.  Reads sp/perm/sel and writes sp2/perm2/sel2
// (sel == nullptr: no selector); fkey/frank are scratch indexed by sorted
// position.  Consecutive receivers then lie close together, so small
// clusters have small bounding boxes.
__global__ __launch_bounds__(kFineWaves * kWave) void k_fine_order(
    const double4 *__restrict__ sp, const int *__restrict__ perm, const uint8_t *__restrict__ sel,
    const int *__restrict__ cs, Geom g, int *__restrict__ fkey, int *__restrict__ frank,
    double4 *__restrict__ sp2, int *__restrict__ perm2, uint8_t *__restrict__ sel2, int keep_max,
    int *__restrict__) {
    __shared__ int hists[kFineWaves][kFineBins];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    int *hist = hists[w];
    for (long long tile = (long long)blockIdx.x * kFineWaves + w; tile < g.nt3;
         tile += (long long)gridDim.x * kFineWaves) {
        const int *c = cs + tile * g.ns3;
        for (int s = 0; s < g.ns3; ++s) {
            const int a0 = c[s], a1 = c[s + 1];
            if (a1 - a0 <= keep_max) continue;   // written in place by k_scatter
            if (a1 - a0 > kFineBig) continue;   // listed by k_big_list
            for (int b = lane; b < kFineBins; b += kWave) hist[b] = 0;
            wave_lds_sync();
            for (int i = a0 + lane; i < a1; i += kWave) {
                const int k = fine_key(sp[i], g);
                fkey[i] = k;
                frank[i] = atomicAdd(&hist[k], 1);
            }
            wave_lds_sync();
            // exclusive scan of the bins: lane l owns bins [l*P, l*P + P)
            constexpr int P = kFineBins / kWave;
            int v[P], sum = 0;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                v[q] = hist[lane * P + q];
                sum += v[q];
            }
            int incl = sum;
            for (int off = 1; off < kWave; off <<= 1) {
                const int y = __shfl_up(incl, off, kWave);
                if (lane >= off) incl += y;
            }
            int run = incl - sum;
#pragma unroll
            for (int q = 0; q < P; ++q) {
                hist[lane * P + q] = run;
                run += v[q];
            }
            wave_lds_sync();
            for (int i = a0 + lane; i < a1; i += kWave) {
                const int dst = a0 + hist[fkey[i]] + frank[i];
                sp2[dst] = sp[i];
                perm2[dst] = perm[i];
                if (sel) sel2[dst] = sel[i];
            }
            wave_lds_sync();
        }
    }
}

// The subtiles holding more than kFineBig particles (big_list[0] counts
// them, zeroed before the launch; the ids follow in any order).
__global__ void k_big_list(const int *__restrict__ cs, long long cells, int *__restrict__ big_list) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    if (cs[c + 1] - cs[c] > kFineBig) big_list[1 + atomicAdd(big_list, 1)] = (int)c;
}

// Fine order of the subtiles holding more than kFineBig particles (listed
// by k_big_list): one block of kFineBins threads per subtile, the same
// counting sort with one bin per thread in the scan.  A single wave would
// take the densest halo cores alone, long after the rest of the grid.
__global__ __launch_bounds__(kFineBins) void k_fine_order_big(
    const double4 *__restrict__ sp, const int *__restrict__ perm, const uint8_t *__restrict__ sel,
    const int *__restrict__ cs, Geom g, int *__restrict__ fkey, int *__restrict__ frank,
    double4 *__restrict__ sp2, int *__restrict__ perm2, uint8_t *__restrict__ sel2,
    const int *__restrict__ big_list) {
    __shared__ int hist[kFineBins];
    __shared__ int lds[kFineBins / kWave];
    const int t = threadIdx.x;
    const int n_big = big_list[0];
    for (int j = blockIdx.x; j < n_big; j += gridDim.x) {
        const int cell = big_list[1 + j];
        const int a0 = cs[cell], a1 = cs[cell + 1];
        hist[t] = 0;
        __syncthreads();
        for (int i = a0 + t; i < a1; i += kFineBins) {
            const int k = fine_key(sp[i], g);
            fkey[i] = k;
            frank[i] = atomicAdd(&hist[k], 1);
        }
        __syncthreads();
        int total;
        const int ex = block_exclusive_scan(hist[t], lds, &total);
        hist[t] = ex;   // every thread has read its own bin in the call above
        __syncthreads();
        for (int i = a0 + t; i < a1; i += kFineBins) {
            const int dst = a0 + hist[fkey[i]] + frank[i];
            sp2[dst] = sp[i];
            perm2[dst] = perm[i];
            if (sel) sel2[dst] = sel[i];
        }
        __syncthreads();
    }
}

// ---- stable order (deterministic mode) ----------------------------------------
//
// The counting sort above ranks the particles of a cell (and of a fine
// sub-cell) by atomics, so their order inside a cell can change between
// calls, and with it the order of every floating-point sum.  The stable path
// sorts the composite key cell << kFineBits | fine sub-cell with an LSD radix
// sort (8-bit digits, stable passes) carrying the particle index; a cell's
// particles then come in (fine sub-cell, index) order, the same on every call,
// and the scatter writes that order directly (no fine-order pass).

constexpr int kFineBits = 9;
static_assert(kFineBins == 1 << kFineBits, "fine sub-cells per subtile");
constexpr int kRsTile = 2048;   // elements per block (one wave) of a radix pass

__global__ void k_rs_keys(const double *__restrict__ pos, int n, Geom g,
                          const int *__restrict__ key, unsigned long long *__restrict__ k64,
                          int *__restrict__ val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double4 p;
    p.x = wrap_coord(pos[3 * (size_t)i], g);
    p.y = wrap_coord(pos[3 * (size_t)i + 1], g);
    p.z = wrap_coord(pos[3 * (size_t)i + 2], g);
    p.w = 0.0;
    k64[i] = ((unsigned long long)(unsigned)key[i] << kFineBits) | (unsigned)fine_key(p, g);
    val[i] = i;
}

// Digit counts of one block's elements, digit-major (hist[d * nblk + b]), so
// that the exclusive scan of hist gives every (digit, block) its first slot.
__global__ __launch_bounds__(kWave) void k_rs_hist(const unsigned long long *__restrict__ k64,
                                                   int n, int shift, int nblk,
                                                   int *__restrict__ hist) {
    __shared__ int cnt[256];
    const int lane = threadIdx.x;
    for (int d = lane; d < 256; d += kWave) cnt[d] = 0;
    wave_lds_sync();
    const size_t base = (size_t)blockIdx.x * kRsTile;
    for (int k = lane; k < kRsTile; k += kWave) {
        const size_t e = base + k;
        if (e < (size_t)n) atomicAdd(&cnt[(int)((k64[e] >> shift) & 255u)], 1);
    }
    wave_lds_sync();
    for (int d = lane; d < 256; d += kWave) hist[(size_t)d * nblk + blockIdx.x] = cnt[d];
}

// Stable scatter of one block's elements by digit: 64 elements at a time in
// index order, each placed after the block's earlier elements of its digit
// (the running slot in LDS) and after the lanes below it with the same digit
// (the lanes whose eight digit-bit ballots all agree with its own).
__global__ __launch_bounds__(kWave) void k_rs_scatter(
    const unsigned long long *__restrict__ kin, const int *__restrict__ vin, int n, int shift,
    int nblk, const int *__restrict__ off, unsigned long long *__restrict__ kout,
    int *__restrict__ vout) {
    __shared__ int run[256];
    const int lane = threadIdx.x;
    for (int d = lane; d < 256; d += kWave) run[d] = off[(size_t)d * nblk + blockIdx.x];
    wave_lds_sync();
    const size_t base = (size_t)blockIdx.x * kRsTile;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int k = 0; k < kRsTile; k += kWave) {
        const size_t e = base + k + lane;
        const bool live = e < (size_t)n;
        const unsigned long long key = live ? kin[e] : 0ull;
        const int v = live ? vin[e] : 0;
        const int d = (int)((key >> shift) & 255u);
        unsigned long long m = __builtin_amdgcn_ballot_w64(live);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long bb = __builtin_amdgcn_ballot_w64(bit);
            m &= bit ? bb : ~bb;
        }
        const int dst = run[d] + __builtin_popcountll(m & below);
        wave_lds_sync();   // every lane has read its digit's slot
        if (live) {
            kout[dst] = key;
            vout[dst] = v;
            if ((m >> lane) == 1ull) run[d] = dst + 1;   // the group's last lane
        }
        wave_lds_sync();
    }
}

// rank[i] = place of particle i inside its cell in the stable order.
__global__ void k_rs_rank(const unsigned long long *__restrict__ k64,
                          const int *__restrict__ val, int n, const int *__restrict__ cell_start,
                          int *__restrict__ rank) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    rank[val[p]] = p - cell_start[(int)(k64[p] >> kFineBits)];
}

// ---- receiver selection and compaction ---------------------------------------

struct Thresholds { uint8_t t[64]; };

__global__ void k_flags(const uint8_t *__restrict__ sel_s, int n, int n_sub, int kind,
                        Thresholds thr, int *__restrict__ flags) {
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)n * n_sub;
    if (idx >= total) return;
    int k = (int)(idx / n);
    int p = (int)(idx - (size_t)k * n);
    int f;
    if (kind == SEL_ALL) f = 1;
    else if (kind == SEL_MASK) f = sel_s[p] != 0;
    else f = sel_s[p] >= thr.t[k];
    flags[idx] = f;
}

__global__ void k_compact(const int *__restrict__ scan, int n, int n_sub, int *__restrict__ act_pos) {
    size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t total = (size_t)n * n_sub;
    if (idx >= total) return;
    int a = scan[idx];
    if (scan[idx + 1] > a) {
        int k = (int)(idx / n);
        act_pos[a] = (int)(idx - (size_t)k * n);
    }
}

__global__ void k_cluster_count(const int *__restrict__ cs, const int *__restrict__ scan, int n,
                                int n_sub, Geom g, int csize, int *__restrict__ ncl) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_sub * g.nt3) return;
    int k = idx / g.nt3;
    int t = idx - k * g.nt3;
    size_t off = (size_t)k * n;
    // scan == nullptr: every particle is a receiver (one subset)
    const int b0 = cs[(size_t)t * g.ns3], b1 = cs[(size_t)(t + 1) * g.ns3];
    int a0 = scan ? scan[off + b0] : b0;
    int a1 = scan ? scan[off + b1] : b1;
    ncl[idx] = (a1 - a0 + csize - 1) / csize;
}

__global__ void k_cluster_write(const int *__restrict__ cs, const int *__restrict__ scan, int n,
                                int n_sub, Geom g, int csize, const int *__restrict__ cl_off,
                                Cluster *__restrict__ clusters) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_sub * g.nt3) return;
    int k = idx / g.nt3;
    int t = idx - k * g.nt3;
    size_t off = (size_t)k * n;
    const int b0 = cs[(size_t)t * g.ns3], b1 = cs[(size_t)(t + 1) * g.ns3];
    int a0 = scan ? scan[off + b0] : b0;
    int a1 = scan ? scan[off + b1] : b1;
    int o = cl_off[idx];
    for (int b = a0; b < a1; b += csize) {
        Cluster c{};
        c.tile = t;
        c.subset = k;
        c.begin = b;
        c.count = min(csize, a1 - b);
        clusters[o++] = c;
    }
}

// ---- work items ------------------------------------------------------------

__global__ void k_item_count(const Cluster *__restrict__ clusters, const int *__restrict__ n_cl,
                             int bound, const int *__restrict__ cs, Geom g, int target, int half,
                             int *__restrict__ item_cnt) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bound) return;
    item_cnt[c] = c < *n_cl ? plan_items(c, clusters[c], cs, g, target, nullptr, 0, half) : 0;
}

// Items of every cluster at their scanned offsets; the cluster count is
// read on the device.
// tot (nullable): the call's receiver, cluster and item totals (three device
// counters) copied to the pinned host array host_tot by the first thread,
// so no launch after the pair kernel is needed for them.
__global__ void k_item_write(const Cluster *__restrict__ clusters, const int *__restrict__ n_cl,
                             int bound, const int *__restrict__ cs, Geom g, int target, int half,
                             const int *__restrict__ item_off, Item *__restrict__ items,
                             const int *tot_recv, const int *tot_items, int *host_tot) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (host_tot && c == 0) {
        host_tot[0] = *tot_recv;
        host_tot[1] = *n_cl;
        host_tot[2] = *tot_items;
    }
    if (c >= bound || c >= *n_cl) return;
    const int off = item_off[c];
    plan_items(c, clusters[c], cs, g, target, items + off,
               item_off[c + 1] - off == 1 ? kItemSole : 0, half);
}

// Deterministic mode: the sums of every cluster with several items, added
// in item order from the items' partial slots (3 doubles per item and
// receiver slot); a cluster's only item stored its sums itself.
__global__ __launch_bounds__(kWave) void k_item_reduce(
    const Cluster *__restrict__ clusters, const int *__restrict__ n_cl,
    const int *__restrict__ item_off, const double *__restrict__ partials, int csize,
    const int *__restrict__ rperm, double *__restrict__ out, long long out_stride) {
    const int nc = *n_cl;
    const int r = threadIdx.x;
    for (int c = blockIdx.x; c < nc; c += gridDim.x) {
        const int i0 = item_off[c], i1 = item_off[c + 1];
        if (i1 - i0 <= 1) continue;
        const Cluster cl = clusters[c];
        if (r >= cl.count) continue;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int it = i0; it < i1; ++it) {
            const double *q = partials + ((size_t)it * csize + r) * 3;
            sx += q[0];
            sy += q[1];
            sz += q[2];
        }
        double *o = out + (long long)cl.subset * out_stride + 3ll * rperm[cl.begin + r];
        o[0] = sx;
        o[1] = sy;
        o[2] = sz;
    }
}

__global__ void k_gather_weights(const double *__restrict__ w, const uint8_t *__restrict__ sel_s,
                                 const int *__restrict__ perm, int n, int fp32,
                                 double4 *__restrict__ wa) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    size_t i = (size_t)perm[p];
    double x = 0, y = 0, z = 0;
    if (!sel_s || sel_s[p]) {   // no selector: all active
        x = w[3 * i];
        y = w[3 * i + 1];
        z = w[3 * i + 2];
    }
    if (fp32) {
        reinterpret_cast<float4 *>(wa)[p] = make_float4((float)x, (float)y, (float)z, 0.0f);
    } else {
        wa[p] = make_double4(x, y, z, 0.0);
    }
}

__device__ inline double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, kWave));
    return v;
}
__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Receivers of each cluster gathered into contiguous arrays (rp / rperm /
// rwa, skipped when rp == nullptr: the receivers are then the sorted
// particles themselves, act_pos == nullptr) and the cluster's bounding box.
// A group of kFinishLanes lanes per cluster, kWave / kFinishLanes clusters
// per wave, kFinishWaves waves per block; each lane takes PPL = csize /
// kFinishLanes receivers, loaded together (the kernel is bound by the
// latency of the two dependent loads, the record and then the receivers, so
// fewer and fuller waves finish sooner), and entries past a cluster's count
// repeat its first receiver.  The cluster count is read on the device, so
// the launch can be sized by an upper bound before the count reaches the
// host.
template <int PPL>
__global__ __launch_bounds__(kFinishWaves * kWave) void k_cluster_finish(
    Cluster *__restrict__ clusters, const int *__restrict__ n_clusters_dev,
    const int *__restrict__ act_pos, const double4 *__restrict__ sp, const int *__restrict__ perm,
    const double4 *__restrict__ wa, double4 *__restrict__ rp, int *__restrict__ rperm,
    double4 *__restrict__ rwa) {
    constexpr int per_wave = kWave / kFinishLanes;
    const int n_clusters = *n_clusters_dev;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = blockIdx.x * kFinishWaves + (int)(threadIdx.x / kWave);
    if (wave * per_wave >= n_clusters) return;   // whole waves leave together
    const int c = wave * per_wave + lane / kFinishLanes;
    const int li = lane & (kFinishLanes - 1);
    const bool have = c < n_clusters;
    double lx = 0.0, ly = 0.0, lz = 0.0, hx = 0.0, hy = 0.0, hz = 0.0;
    if (have) {
        const int begin = clusters[c].begin, count = clusters[c].count;
        double4 x[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int q = li + kFinishLanes * k;
            const int a = begin + (q < count ? q : 0);
            const int p = act_pos ? act_pos[a] : a;
            x[k] = sp[p];
            if (q < count && rp) {
                rp[a] = x[k];
                rperm[a] = perm[p];
                if (rwa) rwa[a] = wa[p];
            }
        }
        lx = hx = x[0].x;
        ly = hy = x[0].y;
        lz = hz = x[0].z;
#pragma unroll
        for (int k = 1; k < PPL; ++k) {
            lx = fmin(lx, x[k].x);
            ly = fmin(ly, x[k].y);
            lz = fmin(lz, x[k].z);
            hx = fmax(hx, x[k].x);
            hy = fmax(hy, x[k].y);
            hz = fmax(hz, x[k].z);
        }
    }
    // min / max over each aligned group of kFinishLanes lanes
#pragma unroll
    for (int off = kFinishLanes >> 1; off > 0; off >>= 1) {
        lx = fmin(lx, __shfl_xor(lx, off, kWave));
        ly = fmin(ly, __shfl_xor(ly, off, kWave));
        lz = fmin(lz, __shfl_xor(lz, off, kWave));
        hx = fmax(hx, __shfl_xor(hx, off, kWave));
        hy = fmax(hy, __shfl_xor(hy, off, kWave));
        hz = fmax(hz, __shfl_xor(hz, off, kWave));
    }
    if (have && li == 0) {
        // only the box: the item kernels may read the other fields meanwhile
        Cluster *o = clusters + c;
        o->lo[0] = lx; o->lo[1] = ly; o->lo[2] = lz;
        o->hi[0] = hx; o->hi[1] = hy; o->hi[2] = hz;
    }
}

// Several int fills in one launch: region blockIdx.y, grid-stride over it.
__global__ void k_fill_multi(FillSet f) {
    const int r = blockIdx.y;
    int *__restrict__ p = f.p[r];
    const size_t n = f.n[r];
    const int v = f.v[r];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

inline unsigned grid_for(size_t n, int block) {
    size_t g = (n + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

hipError_t launch_cluster_finish(Cluster *clusters, const int *n_clusters_dev, size_t bound,
                                 int csize, const int *act_pos, const double4 *sp,
                                 const int *perm, const double4 *wa, double4 *rp, int *rperm,
                                 double4 *rwa, hipStream_t s) {
    if (bound == 0) return hipSuccess;
    const size_t per_block = (size_t)kFinishWaves * (kWave / kFinishLanes);
    if (csize != 8 && csize != 16 && csize != 32 && csize != 64) return hipErrorInvalidValue;
    auto fn = csize == 8    ? k_cluster_finish<1>
              : csize == 16 ? k_cluster_finish<2>
              : csize == 32 ? k_cluster_finish<4>
                            : k_cluster_finish<8>;
    hipLaunchKernelGGL(fn, dim3(grid_for(bound, (int)per_block)), dim3(kFinishWaves * kWave), 0,
                       s, clusters, n_clusters_dev, act_pos, sp, perm, wa, rp, rperm, rwa);
    return hipGetLastError();
}

hipError_t launch_fill_multi(const FillSet &f, hipStream_t s) {
    size_t most = 0;
    for (int r = 0; r < f.count; ++r) most = std::max(most, f.n[r]);
    if (most == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_multi,
                       dim3((unsigned)std::min<size_t>(grid_for(most, 256), 4096), f.count),
                       dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_keys(const double *pos, int n, const Geom &g, int *key, int *rank,
                       int *cell_count, hipStream_t s) {
    if (n == 0) return hipSuccess;
    // the largest block (more particles per global atomic) that still gives
    // every CU a block: 8 particles per thread from N = 2^21, 1 below 2^19
    const size_t per_cu = (size_t)n / (256 * kKeysThreads);
    if (per_cu >= 8)
        hipLaunchKernelGGL(k_keys<8>, dim3(grid_for(n, kKeysThreads * 8)), dim3(kKeysThreads), 0,
                           s, pos, n, g, key, rank, cell_count);
    else if (per_cu >= 4)
        hipLaunchKernelGGL(k_keys<4>, dim3(grid_for(n, kKeysThreads * 4)), dim3(kKeysThreads), 0,
                           s, pos, n, g, key, rank, cell_count);
    else if (per_cu >= 2)
        hipLaunchKernelGGL(k_keys<2>, dim3(grid_for(n, kKeysThreads * 2)), dim3(kKeysThreads), 0,
                           s, pos, n, g, key, rank, cell_count);
    else
        hipLaunchKernelGGL(k_keys<1>, dim3(grid_for(n, kKeysThreads)), dim3(kKeysThreads), 0, s,
                           pos, n, g, key, rank, cell_count);
    return hipGetLastError();
}

size_t scan_block_sums_needed(size_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

size_t scan1_status_needed(size_t n) { return n == 0 ? 1 : (n + kScanTile - 1) / kScanTile; }

hipError_t launch_scan1(const int *in, int *out, size_t n, unsigned long long *status, int *ctr,
                        unsigned long long *stall, int *bsum, hipStream_t s) {
    const size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, out, 0, (size_t)1);
        return hipGetLastError();
    }
    // past a few dozen tiles the blocks running together wait on each
    // other's prefixes in a chain (a rung-batched flag scan of 134M values
    // took 3.9 ms with a one-lane look-back), where three launches take less
    if (nb > (size_t)kScan1MaxTiles) return launch_scan(in, out, n, bsum, s);
    hipLaunchKernelGGL(k_scan_1pass, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n,
                       status, ctr, stall);
    return hipGetLastError();
}

hipError_t launch_scan(const int *in, int *out, size_t n, int *bsum, hipStream_t s) {
    size_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, out, 0, (size_t)1);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, (int)nb, out + n);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n, bsum);
    return hipGetLastError();
}

hipError_t launch_scatter(const double *pos, const double *mass, const uint8_t *sel, int n,
                          const Geom &g, const int *key, const int *rank, const int *cell_start,
                          int fp32, int csize, bool stable, double4 *sp, int *perm,
                          uint8_t *sel_s, double4 *sp2, int *perm2, uint8_t *sel2,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    // stable ranks are already in fine order: every subtile goes straight out
    const int keep_max = stable ? INT_MAX : (csize > kFineMin ? csize : kFineMin);
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, pos, mass, sel, n, g,
                       key, rank, cell_start, fp32, keep_max, sp, perm, sel_s, sp2, perm2, sel2);
    return hipGetLastError();
}

hipError_t launch_big_list(const int *cell_start, const Geom &g, int *big_list, hipStream_t s) {
    // big_list[0] was zeroed on the stream; it holds at most n / kFineBig ids
    const long long cells = (long long)g.nt3 * g.ns3;
    hipLaunchKernelGGL(k_big_list, dim3(grid_for((size_t)cells, 256)), dim3(256), 0, s,
                       cell_start, cells, big_list);
    return hipGetLastError();
}

hipError_t launch_fine_order_medium(const double4 *sp, const int *perm, const uint8_t *sel,
                                    const int *cell_start, const Geom &g, int *fkey, int *frank,
                                    double4 *sp2, int *perm2, uint8_t *sel2, int csize,
                                    hipStream_t s) {
    long long grid = std::min<long long>((g.nt3 + kFineWaves - 1) / kFineWaves, 1ll << 20);
    hipLaunchKernelGGL(k_fine_order, dim3((unsigned)grid), dim3(kFineWaves * kWave), 0, s, sp,
                       perm, sel, cell_start, g, fkey, frank, sp2, perm2, sel2,
                       csize > kFineMin ? csize : kFineMin, (int *)nullptr);
    return hipGetLastError();
}

hipError_t launch_fine_order_big(const double4 *sp, const int *perm, const uint8_t *sel,
                                 const int *cell_start, const Geom &g, int *fkey, int *frank,
                                 double4 *sp2, int *perm2, uint8_t *sel2, int n,
                                 const int *big_list, hipStream_t s) {
    const int big_grid = std::min(n / kFineBig, 256);
    if (big_grid > 0)
        hipLaunchKernelGGL(k_fine_order_big, dim3((unsigned)big_grid), dim3(kFineBins), 0, s, sp,
                           perm, sel, cell_start, g, fkey, frank, sp2, perm2, sel2, big_list);
    return hipGetLastError();
}

hipError_t launch_flags(const uint8_t *sel_s, int n, int n_sub, int kind, const uint8_t *thr_host,
                        int *flags, hipStream_t s) {
    size_t total = (size_t)n * n_sub;
    if (total == 0) return hipSuccess;
    Thresholds thr{};
    if (thr_host)
        for (int k = 0; k < n_sub && k < 64; ++k) thr.t[k] = thr_host[k];
    hipLaunchKernelGGL(k_flags, dim3(grid_for(total, 256)), dim3(256), 0, s, sel_s, n, n_sub, kind,
                       thr, flags);
    return hipGetLastError();
}

// Three device counts into host-visible (pinned) memory: one launch instead
// of a copy per value; read after the stream has been synchronised.
__global__ void k_totals(const int *a, const int *b, const int *c, int *out) {
    if (threadIdx.x == 0) {
        out[0] = *a;
        out[1] = *b;
        out[2] = *c;
    }
}

hipError_t launch_totals(const int *a, const int *b, const int *c, int *host_out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(64), 0, s, a, b, c, host_out);
    return hipGetLastError();
}

hipError_t launch_compact(const int *scan, int n, int n_sub, int *act_pos, hipStream_t s) {
    size_t total = (size_t)n * n_sub;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact, dim3(grid_for(total, 256)), dim3(256), 0, s, scan, n, n_sub,
                       act_pos);
    return hipGetLastError();
}

hipError_t launch_cluster_count(const int *cs, const int *scan, int n, int n_sub, const Geom &g,
                                int csize, int *ncl, hipStream_t s) {
    size_t total = (size_t)n_sub * g.nt3;
    hipLaunchKernelGGL(k_cluster_count, dim3(grid_for(total, 256)), dim3(256), 0, s, cs, scan, n,
                       n_sub, g, csize, ncl);
    return hipGetLastError();
}

hipError_t launch_cluster_write(const int *cs, const int *scan, const int *cl_off, int n,
                                int n_sub, const Geom &g, int csize, Cluster *clusters,
                                hipStream_t s) {
    size_t total = (size_t)n_sub * g.nt3;
    hipLaunchKernelGGL(k_cluster_write, dim3(grid_for(total, 256)), dim3(256), 0, s, cs, scan, n,
                       n_sub, g, csize, cl_off, clusters);
    return hipGetLastError();
}

hipError_t launch_item_count(const Cluster *clusters, const int *n_clusters_dev, int bound,
                             const int *cs, const Geom &g, int target, int half, int *item_cnt,
                             hipStream_t s) {
    if (bound == 0) return hipSuccess;
    hipLaunchKernelGGL(k_item_count, dim3(grid_for(bound, 128)), dim3(128), 0, s, clusters,
                       n_clusters_dev, bound, cs, g, target, half, item_cnt);
    return hipGetLastError();
}

hipError_t launch_item_write(const Cluster *clusters, const int *n_clusters_dev, int bound,
                             const int *cs, const Geom &g, int target, int half,
                             const int *item_off, Item *items, const int *tot_recv,
                             const int *tot_items, int *host_tot, hipStream_t s) {
    if (bound == 0 && !host_tot) return hipSuccess;
    hipLaunchKernelGGL(k_item_write, dim3(grid_for(bound, 128)), dim3(128), 0, s, clusters,
                       n_clusters_dev, bound, cs, g, target, half, item_off, items, tot_recv,
                       tot_items, host_tot);
    return hipGetLastError();
}

// Histogram of particles per tile in 32 bins: bin 0 empty tiles, bin b > 0
// tiles holding [2^(b-1), 2^b) particles (hist zeroed before the launch).
__global__ void k_tile_hist(const int *__restrict__ cs, Geom g, int *__restrict__ hist) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nt3) return;
    const int cnt = cs[(size_t)(t + 1) * g.ns3] - cs[(size_t)t * g.ns3];
    const int b = cnt <= 0 ? 0 : min(31, 32 - __clz(cnt));
    atomicAdd(&hist[b], 1);
}

hipError_t launch_tile_hist(const int *cell_start, const Geom &g, int *hist32, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, hist32, 0, (size_t)32);
    hipLaunchKernelGGL(k_tile_hist, dim3(grid_for((size_t)g.nt3, 256)), dim3(256), 0, s,
                       cell_start, g, hist32);
    return hipGetLastError();
}

hipError_t launch_gather_weights(const double *grad_acc, const uint8_t *sel_s, const int *perm,
                                 int n, int fp32, double4 *wa, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_weights, dim3(grid_for(n, 256)), dim3(256), 0, s, grad_acc, sel_s,
                       perm, n, fp32, wa);
    return hipGetLastError();
}

size_t stable_rank_hist_ints(int n) { return (size_t)256 * ((n + kRsTile - 1) / kRsTile); }

hipError_t launch_stable_ranks(const double *pos, int n, const Geom &g, const int *key,
                               const int *cell_start, unsigned long long *k64a,
                               unsigned long long *k64b, int *va, int *vb, int *hist, int *bsum,
                               int *rank, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int nblk = (n + kRsTile - 1) / kRsTile;
    const long long ncells = (long long)g.nt3 * g.ns3;
    int bits = kFineBits;
    while (bits < 64 && (1ll << (bits - kFineBits)) < ncells) ++bits;
    hipLaunchKernelGGL(k_rs_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, pos, n, g, key, k64a,
                       va);
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kWave), 0, s, k64a, n, shift, nblk, hist);
        hipError_t e = launch_scan(hist, hist, (size_t)256 * nblk, bsum, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kWave), 0, s, k64a, va, n, shift, nblk,
                           hist, k64b, vb);
        std::swap(k64a, k64b);
        std::swap(va, vb);
    }
    hipLaunchKernelGGL(k_rs_rank, dim3(grid_for(n, 256)), dim3(256), 0, s, k64a, va, n,
                       cell_start, rank);
    return hipGetLastError();
}

hipError_t launch_item_reduce(const Cluster *clusters, const int *n_clusters_dev, int bound,
                              const int *item_off, const double *partials, int csize,
                              const int *rperm, double *out, long long out_stride,
                              hipStream_t s) {
    if (bound == 0) return hipSuccess;
    const int grid = std::min(bound, 65536);
    hipLaunchKernelGGL(k_item_reduce, dim3(grid), dim3(kWave), 0, s, clusters, n_clusters_dev,
                       item_off, partials, csize, rperm, out, out_stride);
    return hipGetLastError();
}

}  // namespace p3m
