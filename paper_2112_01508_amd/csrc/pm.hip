// Long-range (PM) half of the P3M gravity: CONCEPT 1.0, section 2.1.3, the
// upper half of eq. p3m_gravity, which runs the PM steps of eq. pm_method
// with the long-range kernel exp(-x_s^2 k^2) / k^2 of eq. ewald_potential:
//
//   sort       counting sort of the particles by lower CIC node
//   deposit    rho_m = sum_j mu_j W(x_m - x_j), CIC weights (eq. W_CIC),
//              cell-centred nodes x_m = h (m + 1/2); runs of one node inside a
//              wavefront are summed first, then FP64 atomics
//   x forward  real lines two at a time as one complex line, radix-2 FFT in
//              LDS, split into the two half spectra (kx = 0 .. n/2)
//   y forward  strided complex FFTs over tiles of adjacent kx columns
//   z          forward FFT, multiply by the kernel, inverse FFT, all in LDS
//              (one pass over HBM instead of three)
//   y inverse
//   x inverse  two half spectra rebuilt into one complex line, inverse FFT,
//              the real and imaginary parts are the two real lines of phi
//   readout    per receiver: 4-point difference (eq. symmetric_diff_4) of phi
//              at the 8 CIC nodes and CIC interpolation (eq. pm_force)
//
// The kernel applied in the z pass is
//   G(k) = 4 pi / h^4 / n^3 * exp(-x_s^2 k^2) / k^2 * prod_d sinc(h k_d / 2)^-4
// (the two CIC deconvolutions of eq. weight_fourier, the 1/n^3 of the
// normalised inverse transform and the prefactor of eq. p3m_gravity folded
// in), G(0) = 0.  It is separable apart from 1/k^2, so two tables of n
// values (per axis index: exp(-x_s^2 k_i^2) sinc^-4 and k_i^2) describe it.
//
// Layouts in HBM: real grids (rho, then phi in the same buffer) are n^3 FP64
// with x fastest, index (z n + y) n + x.  The half-spectrum grid holds
// nh = n/2 + 1 complex FP64 values per (y, z) line at a row stride rs of nh
// rounded up to 8, index (z n + y) rs + kx.
#include <hip/hip_runtime.h>

#include "p3msr_internal.hpp"

namespace p3m {
namespace {

constexpr int kFftThreads = 256;
#ifndef P3M_FFT_TILE
#define P3M_FFT_TILE 2048
#endif
constexpr int kFftTile = P3M_FFT_TILE;   // complex values per workgroup tile (16 B each)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Wrap one coordinate into [0, box) as the oracle does (remainder, then a
// result that rounded up to box itself becomes box - box = 0).
__device__ __forceinline__ double wrap_coord(double x, double box) {
    if (x >= 0.0 && x < box) return x;   // the usual case: already in the box
    double r = fmod(x, box);
    if (r < 0.0) r += box;
    if (r >= box) r -= box;
    return r;
}

// Lower CIC node (in [0, n)) and the weight f of the upper node.
__device__ __forceinline__ int cic_node(double x, double box, double h, int n, double &f) {
    const double u = wrap_coord(x, box) / h - 0.5;
    const double i0 = floor(u);
    f = u - i0;
    return ((int)i0 + n) & (n - 1);
}

// Counting sort of the particles by their lower CIC node (key (z n + y) n + x):
// rank inside the node from an atomic counter, then a scatter to
// start[key] + rank.  The sorted record holds the CIC fractions and mu, so the
// deposit and the readout need neither the positions nor a division.  (Nodes
// are too fine for lanes of a wave to share one often: grouping the lanes by
// node before the atomic, as the cell count does, made this kernel slower.)
__global__ void k_pm_keys(const double *__restrict__ pos, int n_part, int n, double box, double h,
                          int *__restrict__ key, int *__restrict__ rank,
                          int *__restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_part) return;
    double f;
    const int ix = cic_node(pos[3 * (size_t)i], box, h, n, f);
    const int iy = cic_node(pos[3 * (size_t)i + 1], box, h, n, f);
    const int iz = cic_node(pos[3 * (size_t)i + 2], box, h, n, f);
    const int k = (iz * n + iy) * n + ix;
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1);
}

// (Writing only the sorted index here and building the records in sorted
// order with gathered reads took as long: 0.026 + 0.083 ms against 0.114.)
__global__ void k_pm_scatter(const double *__restrict__ pos, const double *__restrict__ mass,
                             const uint8_t *__restrict__ active, int n_part, int n, double box,
                             double h, const int *__restrict__ key, const int *__restrict__ rank,
                             const int *__restrict__ start, double4 *__restrict__ rec,
                             int *__restrict__ nkey, int *__restrict__ perm,
                             uint8_t *__restrict__ recv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_part) return;
    const int k = key[i];
    const int dst = start[k] + rank[i];
    double4 r;
    (void)cic_node(pos[3 * (size_t)i], box, h, n, r.x);
    (void)cic_node(pos[3 * (size_t)i + 1], box, h, n, r.y);
    (void)cic_node(pos[3 * (size_t)i + 2], box, h, n, r.z);
    r.w = mass ? mass[i] : 1.0;
    rec[dst] = r;
    nkey[dst] = k;
    perm[dst] = i;
    recv[dst] = active ? (uint8_t)(active[i] != 0) : (uint8_t)1;
}

// CIC deposit, split by how many particles a source node holds (a node's
// particles are the sorted records start[k] .. start[k+1] - 1).
//
// Sparse source nodes (at most kDenseNode particles) are deposited brick by
// brick: one block owns B^3 grid nodes (B = 16, or 8 on a 16^3 grid), lists
// the particles of the sparse nodes among the (B+1)^3 source nodes that
// reach them (offsets
// 0 or -1 per axis), adds their weights into the brick in LDS and stores the
// brick, so this part needs neither global atomics nor a cleared grid.  In
// the uniform background most nodes hold 0 or 1 particle, where 8 global
// atomics per particle dominated the deposit; a one-thread-per-node gather
// cost as much (16 scattered start[] loads per node).
//
// Dense source nodes: the particles' 8 weights go through global atomics
// after a segmented suffix sum over the wave (lanes that share a node hold
// consecutive records; six shuffle steps leave each run's total with its
// first lane, which alone issues the 8 FP64 atomics).  In halo cores this
// replaces up to 64 serialised atomics on one address by one.  The bricks
// run first; the atomics add on top of them.
constexpr int kDenseNode = 8;

// kBrick^3 nodes per block of kBrickThreads threads; kBrick <= n / 2 keeps the
// (kBrick + 1) source nodes per axis distinct.
template <int kBrick, int kBrickThreads>
__global__ __launch_bounds__(kBrickThreads) void k_pm_deposit_brick(
    const double4 *__restrict__ rec, const int *__restrict__ nkey, const int *__restrict__ start,
    int n, int lg, double *__restrict__ rho) {
    constexpr int kBrickSrc = (kBrick + 1) * (kBrick + 1) * (kBrick + 1);
    constexpr int kBrickPer = (kBrickSrc + kBrickThreads - 1) / kBrickThreads;
    __shared__ double acc[kBrick * kBrick * kBrick];
    __shared__ int src_a[kBrickSrc];          // first record of each listed source node
    __shared__ int pre[kBrickSrc + 1];        // exclusive prefix of their sparse counts
    __shared__ int wsum[kBrickThreads / kWave];
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1), wave = t / kWave;
    const int msk = n - 1;
    const int nb = n / kBrick;
    const int b = blockIdx.x;
    const int x0 = (b % nb) * kBrick, y0 = ((b / nb) % nb) * kBrick, z0 = (b / (nb * nb)) * kBrick;
    for (int j = t; j < kBrick * kBrick * kBrick; j += kBrickThreads) acc[j] = 0.0;
    // source node j = (sz * 9 + sy) * 9 + sx covers (x0 - 1 + sx, y0 - 1 + sy, z0 - 1 + sz)
    int len[kBrickPer];
    int mine = 0;
#pragma unroll
    for (int q = 0; q < kBrickPer; ++q) {
        const int j = t * kBrickPer + q;
        len[q] = 0;
        if (j < kBrickSrc) {
            const int sx = j % (kBrick + 1), sy = (j / (kBrick + 1)) % (kBrick + 1),
                      sz = j / ((kBrick + 1) * (kBrick + 1));
            const size_t g = ((size_t)((z0 - 1 + sz) & msk) * n + ((y0 - 1 + sy) & msk)) * n +
                             ((x0 - 1 + sx) & msk);
            const int a0 = start[g], a1 = start[g + 1];
            src_a[j] = a0;
            len[q] = a1 - a0 <= kDenseNode ? a1 - a0 : 0;
        }
        mine += len[q];
    }
    // block exclusive scan of the per-thread totals
    int incl = mine;
    for (int off = 1; off < kWave; off <<= 1) {
        const int y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    int base = incl - mine, total = 0;
    for (int w = 0; w < kBrickThreads / kWave; ++w) {
        if (w < wave) base += wsum[w];
        total += wsum[w];
    }
#pragma unroll
    for (int q = 0; q < kBrickPer; ++q) {
        const int j = t * kBrickPer + q;
        if (j < kBrickSrc) pre[j] = base;
        base += len[q];
    }
    if (t == 0) pre[kBrickSrc] = total;
    __syncthreads();
    for (int i = t; i < total; i += kBrickThreads) {
        // the listed node holding entry i: the last j with pre[j] <= i
        int lo = 0, hi = kBrickSrc;   // pre[lo] <= i < pre[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= i) lo = mid;
            else hi = mid;
        }
        const int q = src_a[lo] + (i - pre[lo]);
        const double4 r = rec[q];
        const int k = nkey[q];
        const int x = k & msk, y = (k >> lg) & msk, z = k >> (2 * lg);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
            const int tx = (x + cx - x0) & msk, ty = (y + cy - y0) & msk, tz = (z + cz - z0) & msk;
            if (tx < kBrick && ty < kBrick && tz < kBrick) {
                const double wx = cx ? r.x : 1.0 - r.x;
                const double wy = cy ? r.y : 1.0 - r.y;
                const double wz = cz ? r.z : 1.0 - r.z;
                atomicAdd(&acc[(tz * kBrick + ty) * kBrick + tx], r.w * wx * wy * wz);
            }
        }
    }
    __syncthreads();
    for (int j = t; j < kBrick * kBrick * kBrick; j += kBrickThreads) {
        const int tx = j % kBrick, ty = (j / kBrick) % kBrick, tz = j / (kBrick * kBrick);
        rho[((size_t)(z0 + tz) * n + (y0 + ty)) * n + (x0 + tx)] = acc[j];
    }
}

__global__ __launch_bounds__(256) void k_pm_deposit(const double4 *__restrict__ rec,
                                                    const int *__restrict__ nkey,
                                                    const int *__restrict__ start, int n_part,
                                                    double *__restrict__ rho, int n) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    int key = -1 - lane;   // idle and sparse lanes: keys no other lane holds
    bool dense = false;
    double v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = 0.0;
    if (p < n_part) {
        const int k = nkey[p];
        dense = start[k + 1] - start[k] > kDenseNode;
        if (dense) {
            const double4 r = rec[p];
            key = k;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const double wx = (c & 4) ? r.x : 1.0 - r.x;
                const double wy = (c & 2) ? r.y : 1.0 - r.y;
                const double wz = (c & 1) ? r.z : 1.0 - r.z;
                v[c] = r.w * wx * wy * wz;
            }
        }
    }
    // no dense particle in this wave: nothing to add
    if (!__ballot(dense)) return;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int k2 = __shfl_down(key, off, kWave);
        const bool same = lane + off < kWave && k2 == key;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const double o = __shfl_down(v[c], off, kWave);
            if (same) v[c] += o;
        }
    }
    const int prev = __shfl_up(key, 1, kWave);
    if (!dense || (lane > 0 && prev == key)) return;
    const int m = n - 1;
    const int ix = key & m, iy = (key / n) & m, iz = key / (n * n);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const size_t x = (ix + ((c >> 2) & 1)) & m;
        const size_t y = (iy + ((c >> 1) & 1)) & m;
        const size_t z = (iz + (c & 1)) & m;
        atomicAdd(rho + (z * n + y) * n + x, v[c]);
    }
}

// Twiddles tw[m] = exp(-2 pi i m / n), m < n/2, and the kernel tables.
__global__ void k_pm_tables(int n, double box, double x_s, double2 *tw, double *w1,
                            double *k2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n / 2) {
        double s, c;
        sincospi(2.0 * (double)i / (double)n, &s, &c);
        tw[i] = make_double2(c, -s);
    }
    if (i < n) {
        const int hh = i < n / 2 ? i : i - n;
        const double k = 2.0 * M_PI * (double)hh / box;
        double sinc = 1.0;
        if (hh != 0) {
            const double t = (double)hh / (double)n;
            sinc = sinpi(t) / (M_PI * t);
        }
        const double s2 = sinc * sinc;
        k2[i] = k * k;
        w1[i] = exp(-x_s * x_s * k * k) / (s2 * s2);
    }
}

// Copies the n/2 twiddles into LDS (the caller synchronises before use).
template <int N>
__device__ __forceinline__ void stage_twiddles(double2 *tws, const double2 *__restrict__ tw) {
    for (int k = threadIdx.x; k < N / 2; k += kFftThreads) tws[k] = tw[k];
}

// Twiddle exp(-2 pi i m / N) for 0 <= m < N from the half table tw[m < N/2].
template <int N>
__device__ __forceinline__ double2 twiddle(const double2 *tw, int m) {
    if (m < N / 2) return tw[m];
    const double2 w = tw[m - N / 2];
    return make_double2(-w.x, -w.y);
}

// One radix-R Stockham stage (R = 2 or 4) at span Ns: butterfly j reads
// x_q = x[j + q N/R], multiplies x_q by w^(q k) with w = exp(-+2 pi i /
// (R Ns)) and k = j mod Ns, takes the R-point DFT and writes output q to
// (j - k) R + k + q Ns.
template <int N, int LINES, int IS, int LS, bool LANE_J, bool INV, int R>
__device__ __forceinline__ void fft_stage(double2 *buf, const double2 *tw, int Ns) {
    constexpr int NB = LINES * (N / R);
    constexpr int PER = (NB + kFftThreads - 1) / kFftThreads;
    const int t = threadIdx.x;
    const int step = N / (R * Ns);   // twiddle table stride per unit of q k
    double2 y[PER][R];
    int dst[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int bi = t + u * kFftThreads;
        if (NB % kFftThreads == 0 || bi < NB) {
            const int j = LANE_J ? bi % (N / R) : bi / LINES;
            const int l = LANE_J ? bi / (N / R) : bi % LINES;
            const int k = j & (Ns - 1);
            double2 x[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                x[q] = buf[(j + q * (N / R)) * IS + l * LS];
                if (q > 0) {
                    double2 w = twiddle<N>(tw, q * k * step);
                    if (INV) w.y = -w.y;
                    x[q] = cmul(x[q], w);
                }
            }
            if constexpr (R == 2) {
                y[u][0] = make_double2(x[0].x + x[1].x, x[0].y + x[1].y);
                y[u][1] = make_double2(x[0].x - x[1].x, x[0].y - x[1].y);
            } else {
                const double2 a0 = make_double2(x[0].x + x[2].x, x[0].y + x[2].y);
                const double2 a1 = make_double2(x[0].x - x[2].x, x[0].y - x[2].y);
                const double2 a2 = make_double2(x[1].x + x[3].x, x[1].y + x[3].y);
                const double2 d = make_double2(x[1].x - x[3].x, x[1].y - x[3].y);
                // a3 = d * (-i) forward, d * (+i) inverse
                const double2 a3 = INV ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
                y[u][0] = make_double2(a0.x + a2.x, a0.y + a2.y);
                y[u][1] = make_double2(a1.x + a3.x, a1.y + a3.y);
                y[u][2] = make_double2(a0.x - a2.x, a0.y - a2.y);
                y[u][3] = make_double2(a1.x - a3.x, a1.y - a3.y);
            }
            dst[u] = ((j - k) * R + k) * IS + l * LS;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int bi = t + u * kFftThreads;
        if (NB % kFftThreads == 0 || bi < NB) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[dst[u] + q * Ns * IS] = y[u][q];
        }
    }
    __syncthreads();
}

// FFT of `lines` lines of length N held in LDS.  Element (l, i) sits at
// i * IS + l * LS.  Mixed-radix Stockham: radix-4 stages, after one radix-2
// stage when log2 N is odd; the result comes out in natural order without a
// bit reversal.  lane_j: consecutive threads take consecutive j (line-major
// tiles) or consecutive lines (interleaved tiles).
template <int N, int LINES, int IS, int LS, bool LANE_J, bool INV>
__device__ __forceinline__ void lds_fft(double2 *buf, const double2 *tw) {
    constexpr int LOG = __builtin_ctz(N);
    int Ns = 1;
    if constexpr (LOG % 2 == 1) {
        fft_stage<N, LINES, IS, LS, LANE_J, INV, 2>(buf, tw, 1);
        Ns = 2;
    }
#pragma unroll 1
    for (; Ns < N; Ns *= 4) fft_stage<N, LINES, IS, LS, LANE_J, INV, 4>(buf, tw, Ns);
}

// Half-spectrum rows hold NH = N/2 + 1 values, stored with a stride rounded
// up to 8 complex values (128 B) so that column tiles start on cache lines.
template <int N>
struct Row {
    static constexpr int kNH = N / 2 + 1;
    static constexpr int kStride = (kNH + 7) & ~7;
};

template <int N>
struct XTile {
    static constexpr int kLines = (kFftTile / N) < (N * N / 2) ? (kFftTile / N) : (N * N / 2);
};

// x forward: real lines 2p, 2p+1 of rho as the real and imaginary parts of
// one complex line; after the FFT Z, A_k = (Z_k + conj Z_{N-k}) / 2 and
// B_k = -i (Z_k - conj Z_{N-k}) / 2 are the spectra of the two real lines.
template <int N>
__global__ __launch_bounds__(kFftThreads) void k_fft_x_fwd(const double *__restrict__ rho,
                                                           double2 *__restrict__ spec,
                                                           const double2 *__restrict__ tw) {
    constexpr int P = XTile<N>::kLines;     // complex lines per tile
    constexpr int NH = N / 2 + 1;
    __shared__ double2 buf[P * N];
    __shared__ double2 tws[N / 2];
    stage_twiddles<N>(tws, tw);
    const size_t line0 = (size_t)blockIdx.x * 2 * P;   // first real line of the tile
    const double *src = rho + line0 * N;
    double *bufd = reinterpret_cast<double *>(buf);
    for (int e = threadIdx.x; e < 2 * P * N; e += kFftThreads) {
        const int r = e / N, i = e % N;
        bufd[2 * ((r >> 1) * N + i) + (r & 1)] = src[e];
    }
    __syncthreads();
    lds_fft<N, P, 1, N, true, false>(buf, tws);
    double2 *dst = spec + line0 * Row<N>::kStride;
    // both half spectra of a line pair from one read of Z_k and Z_{N-k}
    for (int e = threadIdx.x; e < P * NH; e += kFftThreads) {
        const int p = e / NH, k = e % NH;
        const double2 z = buf[p * N + k];
        const double2 zc = buf[p * N + ((N - k) & (N - 1))];   // enters conjugated
        dst[(size_t)(2 * p) * Row<N>::kStride + k] =
            make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        dst[(size_t)(2 * p + 1) * Row<N>::kStride + k] =
            make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
}

// x inverse: Z_k = A_k + i B_k (k <= N/2), conj(A_{N-k}) + i conj(B_{N-k})
// above; the inverse FFT of Z holds line 2p in its real part and line 2p+1
// in its imaginary part.
template <int N>
__global__ __launch_bounds__(kFftThreads) void k_fft_x_inv(const double2 *__restrict__ spec,
                                                           double *__restrict__ phi,
                                                           const double2 *__restrict__ tw) {
    constexpr int P = XTile<N>::kLines;
    constexpr int NH = N / 2 + 1;
    __shared__ double2 buf[P * N];
    __shared__ double2 tws[N / 2];
    stage_twiddles<N>(tws, tw);
    const size_t line0 = (size_t)blockIdx.x * 2 * P;
    const double2 *src = spec + line0 * Row<N>::kStride;
    for (int e = threadIdx.x; e < P * N; e += kFftThreads) {
        const int p = e / N, k = e % N;
        const bool lo = k <= N / 2;
        const int kk = lo ? k : N - k;
        const double2 a = src[(size_t)(2 * p) * Row<N>::kStride + kk];
        const double2 b = src[(size_t)(2 * p + 1) * Row<N>::kStride + kk];
        buf[e] = lo ? make_double2(a.x - b.y, a.y + b.x) : make_double2(a.x + b.y, b.x - a.y);
    }
    __syncthreads();
    lds_fft<N, P, 1, N, true, true>(buf, tws);
    double *dst = phi + line0 * N;
    const double *bufd = reinterpret_cast<const double *>(buf);
    for (int e = threadIdx.x; e < 2 * P * N; e += kFftThreads) {
        const int r = e / N, i = e % N;
        dst[e] = bufd[2 * ((r >> 1) * N + i) + (r & 1)];
    }
}

template <int N>
struct STile {
    // 4..16 adjacent columns: rows are read at least 64 B at a time
    static constexpr int kRaw = kFftTile / N;
    static constexpr int kCols = kRaw < 4 ? 4 : (kRaw > 16 ? 16 : kRaw);
};

// Strided passes over tiles of C adjacent kx columns.  AXIS 1 (y): blockIdx.y
// is z, elements step by the row stride.  AXIS 2 (z): blockIdx.y is y,
// elements step by N row strides.  CONV: forward FFT, multiply by the kernel,
// inverse FFT.
template <int N, int AXIS, int MODE>   // MODE 0 forward, 1 inverse, 2 convolve
__global__ __launch_bounds__(kFftThreads) void k_fft_strided(double2 *__restrict__ spec,
                                                             const double2 *__restrict__ tw,
                                                             const double *__restrict__ w1,
                                                             const double *__restrict__ k2,
                                                             double scale) {
    constexpr int C = STile<N>::kCols;
    constexpr int NH = N / 2 + 1;
    __shared__ double2 buf[C * N];
    __shared__ double2 tws[N / 2];
    stage_twiddles<N>(tws, tw);
    const int kx0 = blockIdx.x * C;
    const int other = blockIdx.y;   // z for the y pass, y for the z pass
    constexpr size_t RS = Row<N>::kStride;
    const size_t base = AXIS == 1 ? (size_t)other * N * RS + kx0 : (size_t)other * RS + kx0;
    const size_t step = AXIS == 1 ? RS : (size_t)N * RS;
    const int ncol = NH - kx0 < C ? NH - kx0 : C;
    for (int e = threadIdx.x; e < C * N; e += kFftThreads) {
        const int c = e % C, i = e / C;
        buf[e] = c < ncol ? spec[base + (size_t)i * step + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (MODE == 1) {
        lds_fft<N, C, C, 1, false, true>(buf, tws);
    } else {
        lds_fft<N, C, C, 1, false, false>(buf, tws);
    }
    if (MODE == 2) {
        // element (c, kz) of column kx = kx0 + c on the line ky = other
        const double wy = w1[other], ky2 = k2[other];
        for (int e = threadIdx.x; e < C * N; e += kFftThreads) {
            const int c = e % C, kz = e / C;
            const int kx = kx0 + c;
            if (c < ncol) {
                const double kk = k2[kx] + ky2 + k2[kz];
                const double g = kk > 0.0 ? scale * (w1[kx] * wy * w1[kz]) / kk : 0.0;
                buf[e] = make_double2(buf[e].x * g, buf[e].y * g);
            }
        }
        __syncthreads();
        lds_fft<N, C, C, 1, false, true>(buf, tws);
    }
    for (int e = threadIdx.x; e < C * N; e += kFftThreads) {
        const int c = e % C, i = e / C;
        if (c < ncol) spec[base + (size_t)i * step + c] = buf[e];
    }
}

// Readout: per receiver, the 4-point difference of phi along each axis at
// the 8 CIC nodes and their CIC-weighted sum.  Along x the six values
// phi[i0-2 .. i0+3] of each (y, z) node pair give D4 at i0 and i0 + 1; the
// same for y and z.
__device__ __forceinline__ double d4_at(const double *v) {
    // v[0..4] = phi[m-2 .. m+2]
    return (v[0] - 8.0 * v[1] + 8.0 * v[3] - v[4]) / 12.0;
}

// (Staging phi per brick in LDS and reading the stencils from there was
// slower: 241 us with 16^3 bricks and 275 us with 8^3 against 216 us for
// this per-particle gather on clustered128's 256^3 grid.)
__global__ void k_pm_readout(const double4 *__restrict__ rec, const int *__restrict__ nkey,
                             const int *__restrict__ perm, const uint8_t *__restrict__ recv,
                             int n_part, const double *__restrict__ phi, int n,
                             double *__restrict__ acc) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_part) return;
    const size_t i = (size_t)perm[p];
    if (!recv[p]) {
        acc[3 * i] = 0.0;
        acc[3 * i + 1] = 0.0;
        acc[3 * i + 2] = 0.0;
        return;
    }
    const double4 r = rec[p];
    const int key = nkey[p];
    const int m = n - 1;
    const int i0[3] = {key & m, (key / n) & m, key / (n * n)};
    const double f[3] = {r.x, r.y, r.z};
    const size_t str[3] = {1, (size_t)n, (size_t)n * n};
    double out[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // the two axes other than d
        const int a = d == 0 ? 1 : 0;
        const int b = d == 2 ? 1 : 2;
        double sum = 0.0;
#pragma unroll
        for (int ca = 0; ca < 2; ++ca) {
            const double wa = ca ? f[a] : 1.0 - f[a];
            const size_t oa = (size_t)((i0[a] + ca) & m) * str[a];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const double wb = cb ? f[b] : 1.0 - f[b];
                const size_t ob = (size_t)((i0[b] + cb) & m) * str[b];
                double v[6];
#pragma unroll
                for (int s = 0; s < 6; ++s)
                    v[s] = phi[oa + ob + (size_t)((i0[d] - 2 + s + n) & m) * str[d]];
                const double line = (1.0 - f[d]) * d4_at(v) + f[d] * d4_at(v + 1);
                sum += wa * wb * line;
            }
        }
        out[d] = sum;
    }
    acc[3 * i] = out[0];
    acc[3 * i + 1] = out[1];
    acc[3 * i + 2] = out[2];
}

template <int N>
hipError_t launch_fft_chain_n(const PmArgs &a, hipStream_t s, hipEvent_t *ev) {
    constexpr int NH = N / 2 + 1;
    constexpr int P = XTile<N>::kLines;
    constexpr int C = STile<N>::kCols;
    const int x_blocks = (N * N) / (2 * P);
    const dim3 s_grid((NH + C - 1) / C, N);
    hipError_t e;
    k_fft_x_fwd<N><<<x_blocks, kFftThreads, 0, s>>>(a.real, a.spec, a.tw);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    k_fft_strided<N, 1, 0><<<s_grid, kFftThreads, 0, s>>>(a.spec, a.tw, a.w1, a.k2, a.scale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    k_fft_strided<N, 2, 2><<<s_grid, kFftThreads, 0, s>>>(a.spec, a.tw, a.w1, a.k2, a.scale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    k_fft_strided<N, 1, 1><<<s_grid, kFftThreads, 0, s>>>(a.spec, a.tw, a.w1, a.k2, a.scale);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    k_fft_x_inv<N><<<x_blocks, kFftThreads, 0, s>>>(a.spec, a.real, a.tw);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pm_tables(int n, double box, double x_s, double2 *tw, double *w1, double *k2,
                            hipStream_t s) {
    k_pm_tables<<<(n + 255) / 256, 256, 0, s>>>(n, box, x_s, tw, w1, k2);
    return hipGetLastError();
}

hipError_t launch_pm_sort(const double *pos, const double *mass, const uint8_t *active,
                          int n_part, int n, double box, double h, int *key, int *rank,
                          int *count, int *bsum, double4 *rec, int *nkey, int *perm,
                          uint8_t *recv, hipStream_t s) {
    const size_t cells = (size_t)n * n * n;
    hipError_t e;
    if ((e = launch_fill_i32(count, 0, cells + 1, s)) != hipSuccess) return e;
    const unsigned grid = (unsigned)((n_part + 255) / 256);
    if (n_part > 0) {
        k_pm_keys<<<grid, 256, 0, s>>>(pos, n_part, n, box, h, key, rank, count);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_part == 0) return hipSuccess;
    // start[k] = first sorted index of node k
    if ((e = launch_scan(count, count, cells, bsum, s)) != hipSuccess) return e;
    k_pm_scatter<<<grid, 256, 0, s>>>(pos, mass, active, n_part, n, box, h, key, rank, count, rec,
                                      nkey, perm, recv);
    return hipGetLastError();
}

hipError_t launch_pm_deposit(const double4 *rec, const int *nkey, const int *start, int n_part,
                             double *rho, int n, hipStream_t s) {
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    if (n >= 32) {
        const size_t nb = (size_t)n / 16;
        k_pm_deposit_brick<16, 1024><<<(unsigned)(nb * nb * nb), 1024, 0, s>>>(rec, nkey, start,
                                                                              n, lg, rho);
    } else {
        const size_t nb = (size_t)n / 8;
        k_pm_deposit_brick<8, 256><<<(unsigned)(nb * nb * nb), 256, 0, s>>>(rec, nkey, start, n,
                                                                           lg, rho);
    }
    hipError_t e;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_part == 0) return hipSuccess;
    k_pm_deposit<<<(unsigned)((n_part + 255) / 256), 256, 0, s>>>(rec, nkey, start, n_part, rho, n);
    return hipGetLastError();
}

hipError_t launch_pm_fft_chain(const PmArgs &a, hipStream_t s, hipEvent_t *ev) {
    switch (a.n) {
        case 16: return launch_fft_chain_n<16>(a, s, ev);
        case 32: return launch_fft_chain_n<32>(a, s, ev);
        case 64: return launch_fft_chain_n<64>(a, s, ev);
        case 128: return launch_fft_chain_n<128>(a, s, ev);
        case 256: return launch_fft_chain_n<256>(a, s, ev);
        case 512: return launch_fft_chain_n<512>(a, s, ev);
        case 1024: return launch_fft_chain_n<1024>(a, s, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pm_readout(const double4 *rec, const int *nkey, const int *perm,
                             const uint8_t *recv, int n_part, const double *phi, int n,
                             double *acc, hipStream_t s) {
    if (n_part == 0) return hipSuccess;
    k_pm_readout<<<(unsigned)((n_part + 255) / 256), 256, 0, s>>>(rec, nkey, perm, recv, n_part,
                                                                 phi, n, acc);
    return hipGetLastError();
}

}  // namespace p3m
