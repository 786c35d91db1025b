// Short-range pair kernels: forward force and its adjoint, FP32 and FP64.
//
// Force (section 2.1.3, lower half of eq. p3m_gravity, no softening):
//   a_i = - sum_{j != i, r < r_cut} mu_j g(u) r_ij / r^3,  u = r / (2 x_s),
//   g(u) = erfc(u) + (2/sqrt(pi)) u exp(-u^2),
// with r_ij taken to the nearest periodic image n'.  The image is fixed per
// neighbour tile (section 2.1.3, "Other optimisations": n' follows from the
// tile pair), and the zero-shift case runs in its own loop.
//
// Traversal (one wavefront per work item, persistent grid): the lanes hold
// the <= 64 receivers of one cluster in registers; for each neighbour tile
// of the item the lanes test one subtile each against the cluster's
// bounding box (the subtile-pair culling of section 2.1.3, "Subtiles", done
// against the receivers' actual extent), a ballot gives the surviving
// subtiles, and consecutive survivors merge into supplier ranges.  Supplier
// particles are streamed by every lane; when a cluster holds fewer than 64
// receivers the wave carries G = 64 / count copies of it and each copy walks
// a different stride of the supplier range, so lanes are not left idle.
//
// Precision: the separation r_ij, the squared distance and the cut-off
// test are FP64 and bitwise the same as a plain FP64 evaluation, so both
// paths accept exactly the same pairs.  The kernel shape uses the identity
// g(u)/r^3 = r^-3 + H(u^2) / (2 x_s)^3 (g - 1 has only odd powers of u from
// u^3 on): the FP32 path with hardware rsqrt and a degree-9 polynomial, the
// FP64 path with an FP64 rsqrt and a degree-17 polynomial (and its
// derivative for the adjoint).  The FP32 adjoint uses hardware rsqrt and
// exp2 and a degree-9 polynomial for erfcx(u) + 2u/sqrt(pi).  Accumulation
// is FP64 everywhere.
#include "p3msr_internal.hpp"
#include "gpoly.inc"

namespace p3m {

namespace {

__device__ inline unsigned long long ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of lanes of the wave whose squared distance r2 passes the cut-off
// test 0 < r2 < rc2.  The ballot of a single compare is that compare's own
// lane mask, so with one ballot per compare the count is two scalar ANDs and
// a population count on the scalar unit, and no vector instruction.  Called
// in wave-uniform control flow only (all 64 lanes active), where the running
// total stays wave-uniform.  The loops below sum these counts in 32 bits
// (one scalar add per step) and add the sum to the wave's 64-bit total once
// per supplier range or list.
__device__ __forceinline__ unsigned count_pass(double r2, double rc2) {
    return (unsigned)__builtin_popcountll(ballot64(r2 < rc2) & ballot64(r2 > 0.0));
}

__device__ inline float q_poly(float v) {
    float q = kGpoly[P3M_GPOLY_DEGREE];
#pragma unroll
    for (int k = P3M_GPOLY_DEGREE - 1; k >= 0; --k) q = fmaf(q, v, kGpoly[k]);
    return q;
}

__device__ inline float h_poly(float v) {
    float h = kHpoly[P3M_HPOLY_DEGREE];
#pragma unroll
    for (int k = P3M_HPOLY_DEGREE - 1; k >= 0; --k) h = fmaf(h, v, kHpoly[k]);
    return h;
}

// FP64 H and, optionally, dH/dv from one Horner pass; the coefficients come
// from the kernel arguments (SGPRs) so each step is one v_fma_f64.
// 1/sqrt(x) in FP64 for a positive normal x (the pair loop's 0 < r^2 < r_cut^2):
// the hardware estimate y0 and one step of the series
// (1 - e)^(-1/2) = 1 + e/2 + 3 e^2 / 8 + ...,  e = 1 - x y0^2,
// which triples the estimate's correct bits.  Zero, infinite and subnormal
// inputs need no handling here.
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

__device__ inline double h64(double v, const double *c) {
    double h = c[P3M_H64_DEGREE];
#pragma unroll
    for (int k = P3M_H64_DEGREE - 1; k >= 0; --k) h = fma(h, v, c[k]);
    return h;
}
__device__ inline double h64_d(double v, const double *c, double &dh) {
    double h = c[P3M_H64_DEGREE], d = 0.0;
#pragma unroll
    for (int k = P3M_H64_DEGREE - 1; k >= 0; --k) {
        d = fma(d, v, h);
        h = fma(h, v, c[k]);
    }
    dh = d;
    return h;
}

__device__ inline float mu_f32(double w) {
    return __uint_as_float((unsigned int)(unsigned long long)__double_as_longlong(w));
}

// Squared distance of the cut-off test, rounded as fma(dz, dz, fma(dy, dy,
// dx * dx)): three instructions instead of five, and the rounding every
// implementation of the test uses, so accept / reject decisions near r_cut
// are the same everywhere.
__device__ inline double dist2(double dx, double dy, double dz) {
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// ---- B-spline softening (section 2.1.1, eq. bspline_force) --------------------

// For r < eps_b the pair factor g(u)/r^3 = r^-3 + c3 H(t) of the point-particle
// force gains the softening bracket |r|_B^-3 - r^-3 of eq. p3m_gravity, so it
// becomes c3 H(t) + |r|_B^-3.  With x = r / eps_b and ks3 = 32 / eps_b^3:
//   x < 1/2:  |r|_B^-3 = ks3 (x^3 - 6/5 x^2 + 1/3)
//   x >= 1/2: |r|_B^-3 = ks3 (-x^3/3 + 6/5 x^2 - 3/2 x + 2/3) - r^-3 / 15
// (the x^-3 / 480 term of eq. bspline_force times ks3 is r^-3 / 15).
__device__ inline double bspline_m3(double x, double ri3, const Geom &g) {
    if (x < 0.5) return g.ks3 * fma(x * x, x - 1.2, 1.0 / 3.0);
    return g.ks3 * fma(fma(fma(-1.0 / 3.0, x, 1.2), x, -1.5), x, 2.0 / 3.0) - ri3 * (1.0 / 15.0);
}

// -(d|r|_B^-3 / dr) / r, ks5 = 32 / eps_b^5:
//   x < 1/2:  ks5 (12/5 - 3 x)
//   x >= 1/2: ks5 (x - 12/5 + 3/2 eps_b / r) - r^-5 / 5
__device__ inline double bspline_m3_c(double x, double ri, double ri5, const Geom &g) {
    if (x < 0.5) return g.ks5 * (2.4 - 3.0 * x);
    return g.ks5 * (x - 2.4 + 1.5 * g.eps_b * ri) - ri5 * 0.2;
}

// ---- per-pair bodies ---------------------------------------------------------

// Forward, FP32 shape: g(u)/r^3 = r^-3 + H(t) / (2 x_s)^3 with t = u^2 (one
// hardware rsqrt and one polynomial, no exponential).  UNIT: every mass is 1.
// SOFT: pairs inside the softening length take c3 H(t) + |r|_B^-3, with the
// softening term in FP64 (it cancels to a few percent of its parts near
// r = eps_b).
//
// TAB (point particles only): H is looked up instead of evaluated, in a table
// over r^2 in [0, r_cut^2) held in LDS - the paper's 1D table indexed by r^2
// (section 2.1.3, "Other optimisations"), here of the smooth part only, since
// the r^-3 part diverges at r = 0 and costs one rsqrt.  SHAPE_TAB_NGP: the
// value of the bin (nearest grid point); SHAPE_TAB_LINEAR: linear
// interpolation between the bin's nodes.
template <bool UNIT, bool SOFT, int TAB = SHAPE_POLY>
struct FwdF32 {
    static constexpr bool kNeedW = !UNIT;
    static constexpr bool kHasW = false;   // no per-supplier adjoint weight
    using WT = float;
    double ax = 0.0, ay = 0.0, az = 0.0;
    const float *tab = nullptr;            // the LDS copy of the table (TAB != 0)
    __device__ __forceinline__ void pair_w(double dx, double dy, double dz, double r2,
                                           const double4 &pj, const WT &, const PairArgs &a) {
        pair(dx, dy, dz, r2, pj, 0, a);
    }
    __device__ __forceinline__ void pair(double dx, double dy, double dz, double r2,
                                         const double4 &pj, int, const PairArgs &a) {
        const Geom &g = a.g;
        const float r2f = (float)r2;
        const float ri = __builtin_amdgcn_rsqf(r2f);
        float h;
        if constexpr (TAB == SHAPE_TAB_NGP) {
            const int k = min((int)(r2f * a.tab_scale), a.tab_n - 1);
            h = tab[k];
        } else if constexpr (TAB == SHAPE_TAB_LINEAR) {
            const float x = r2f * a.tab_scale;
            const int k = min((int)x, a.tab_n - 1);
            const float2 e = reinterpret_cast<const float2 *>(tab)[k];
            h = fmaf(e.y, x - (float)k, e.x);
        } else {
            h = h_poly(fmaf(r2f, g.c2f, -P3M_HPOLY_T0));
        }
        const float ri3 = ri * ri * ri;
        double sd;
        if (SOFT && r2 < g.eps_b2) {
            const double x = (double)(r2f * ri * g.inv_eps_bf);
            sd = (double)(g.c3f * h) + bspline_m3(x, (double)ri3, g);
            if (!UNIT) sd *= (double)mu_f32(pj.w);
        } else {
            const float sh = fmaf(g.c3f, h, ri3);
            sd = (double)(UNIT ? sh : mu_f32(pj.w) * sh);
        }
        ax = fma(-sd, dx, ax);
        ay = fma(-sd, dy, ay);
        az = fma(-sd, dz, az);
    }
};

// Forward, FP64 shape: the same identity g(u)/r^3 = r^-3 + H(t) / (2 x_s)^3
// with an FP64 rsqrt and a degree-17 polynomial (error 1.5e-15 in g).
template <bool UNIT, bool SOFT>
struct FwdF64 {
    static constexpr bool kNeedW = !UNIT;
    static constexpr bool kHasW = false;   // no per-supplier adjoint weight
    using WT = float;
    double ax = 0.0, ay = 0.0, az = 0.0;
    __device__ __forceinline__ void pair_w(double dx, double dy, double dz, double r2,
                                           const double4 &pj, const WT &, const PairArgs &a) {
        pair(dx, dy, dz, r2, pj, 0, a);
    }
    __device__ __forceinline__ void pair(double dx, double dy, double dz, double r2,
                                         const double4 &pj, int, const PairArgs &a) {
        const double ri = rsqrt_pos(r2);
        const double h = h64(fma(r2, a.g.c2, -P3M_H64_T0), a.g.h64);
        const double ri3 = ri * ri * ri;
        double sh;
        if (SOFT && r2 < a.g.eps_b2) sh = fma(a.g.c3, h, bspline_m3(r2 * ri * a.g.inv_eps_b, ri3, a.g));
        else sh = fma(a.g.c3, h, ri3);
        const double s = UNIT ? sh : pj.w * sh;
        ax -= s * dx;
        ay -= s * dy;
        az -= s * dz;
    }
};

// Adjoint: grad_k -= J(r_kj) (mu_j wa_k - mu_k wa_j), wa = w * [active],
// J = phi I - c r r^T with phi = g / r^3 = r^-3 + c3 H(t) and
// c = -(dphi/dr)/r = 3 g / r^5 + exp(-u^2) / (2 sqrt(pi) x_s^3 r^2)
//   = 3 r^-5 - 2 c2 c3 H'(t)   (t = r^2 c2).
// Inside the softening length phi = c3 H(t) + |r|_B^-3 and
// c = -2 c2 c3 H'(t) - (d|r|_B^-3/dr) / r.
template <bool SOFT>
struct BwdF64 {
    static constexpr bool kNeedW = true;
    static constexpr bool kHasW = true;    // supplier weight w_j [j active]
    using WT = double4;
    double ax = 0.0, ay = 0.0, az = 0.0;
    double wkx, wky, wkz, muk;
    __device__ __forceinline__ static WT weight(const PairArgs &a, int j) { return a.wa[j]; }
    __device__ __forceinline__ void pair(double dx, double dy, double dz, double r2,
                                         const double4 &pj, int j, const PairArgs &a) {
        pair_w(dx, dy, dz, r2, pj, a.wa[j], a);   // j may be wave-uniform or per lane
    }
    __device__ __forceinline__ void pair_w(double dx, double dy, double dz, double r2,
                                           const double4 &pj, const double4 &wj,
                                           const PairArgs &a) {
        double vx = pj.w * wkx - muk * wj.x;
        double vy = pj.w * wky - muk * wj.y;
        double vz = pj.w * wkz - muk * wj.z;
        const double ri = rsqrt_pos(r2);
        const double ri2 = ri * ri;
        double dh;
        const double h = h64_d(fma(r2, a.g.c2, -P3M_H64_T0), a.g.h64, dh);
        double phi, c;
        if (SOFT && r2 < a.g.eps_b2) {
            const double x = r2 * ri * a.g.inv_eps_b;
            phi = fma(a.g.c3, h, bspline_m3(x, ri2 * ri, a.g));
            c = fma(-2.0 * a.g.c2 * a.g.c3, dh, bspline_m3_c(x, ri, ri2 * ri2 * ri, a.g));
        } else {
            phi = fma(a.g.c3, h, ri2 * ri);
            c = fma(3.0 * ri2 * ri2, ri, -2.0 * a.g.c2 * a.g.c3 * dh);
        }
        double rv = dx * vx + dy * vy + dz * vz;
        ax -= phi * vx - c * rv * dx;
        ay -= phi * vy - c * rv * dy;
        az -= phi * vz - c * rv * dz;
    }
};

// FP32 adjoint: phi and c from hardware exp2 and rsqrt with a polynomial for
// erfcx(u) + 2u/sqrt(pi).  Inside the softening length phi - r^-3 would
// cancel in FP32, so those pairs take the FP64 H form of BwdF64.
template <bool SOFT>
struct BwdF32 {
    static constexpr bool kNeedW = true;
    static constexpr bool kHasW = true;    // supplier weight w_j [j active], FP32
    using WT = float4;
    double ax = 0.0, ay = 0.0, az = 0.0;
    float wkx, wky, wkz, muk;
    __device__ __forceinline__ static WT weight(const PairArgs &a, int j) {
        return reinterpret_cast<const float4 *>(a.wa)[j];
    }
    __device__ __forceinline__ void pair(double dx, double dy, double dz, double r2,
                                         const double4 &pj, int j, const PairArgs &a) {
        pair_w(dx, dy, dz, r2, pj, weight(a, j), a);
    }
    __device__ __forceinline__ void pair_w(double dx, double dy, double dz, double r2,
                                           const double4 &pj, const float4 &wj,
                                           const PairArgs &a) {
        const Geom &g = a.g;
        const float muj = mu_f32(pj.w);
        float vx = muj * wkx - muk * wj.x;
        float vy = muj * wky - muk * wj.y;
        float vz = muj * wkz - muk * wj.z;
        if (SOFT && r2 < g.eps_b2) {
            const double ri = rsqrt_pos(r2);
            const double ri2 = ri * ri;
            const double x = r2 * ri * g.inv_eps_b;
            double dh;
            const double h = h64_d(fma(r2, g.c2, -P3M_H64_T0), g.h64, dh);
            const double phi = fma(g.c3, h, bspline_m3(x, ri2 * ri, g));
            const double c = fma(-2.0 * g.c2 * g.c3, dh, bspline_m3_c(x, ri, ri2 * ri2 * ri, g));
            const double rv = dx * vx + dy * vy + dz * vz;
            ax -= phi * vx - c * rv * dx;
            ay -= phi * vy - c * rv * dy;
            az -= phi * vz - c * rv * dz;
            return;
        }
        float r2f = (float)r2;
        float ri = __builtin_amdgcn_rsqf(r2f);
        float ri2 = ri * ri;
        float v = fmaf(r2f * ri, g.k1f, -P3M_GPOLY_C0);
        float e = __builtin_amdgcn_exp2f((float)(r2 * g.k2));
        float gu = e * q_poly(v);
        float phi = gu * ri2 * ri;
        float c = ri2 * fmaf(3.0f, phi, g.kbf * e);
        float fx = (float)dx, fy = (float)dy, fz = (float)dz;
        float rv = fx * vx + fy * vy + fz * vz;
        float crv = c * rv;
        ax -= (double)fmaf(phi, vx, -crv * fx);
        ay -= (double)fmaf(phi, vy, -crv * fy);
        az -= (double)fmaf(phi, vz, -crv * fz);
    }
};

// ---- supplier range loop ------------------------------------------------------

// Pointer into the constant address space: loads through it at wave-uniform
// addresses become scalar loads into SGPRs.  The supplier array is not
// written by the pair kernels.
template <class T>
using ConstPtr = const __attribute__((address_space(4))) T *;

__device__ __forceinline__ double4 load_uniform(const double4 *base, int j) {
    ConstPtr<double> q = (ConstPtr<double>)base + 4 * (long long)j;
    return make_double4(q[0], q[1], q[2], q[3]);
}

// One receiver lane against one supplier: the separation (with the tile's
// periodic image), the squared distance and the strict cut-off test in FP64,
// then the pair body.  n_lane counts this lane's accepted pairs: this loop
// reads its suppliers through the scalar unit, which a scalar count would
// load further (measured 1-2 % slower than the vector add here).
template <bool SHIFT, class Body>
__device__ __forceinline__ void test_pair(Body &body, double xi, double yi, double zi,
                                          const double4 &pj, int j, bool valid, double shx,
                                          double shy, double shz, const PairArgs &a,
                                          int &n_lane) {
    double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
    if (SHIFT) {
        dx -= shx;
        dy -= shy;
        dz -= shz;
    }
    const double r2 = dist2(dx, dy, dz);
    if (valid & (r2 < a.g.rc2) & (r2 > 0.0)) {
        ++n_lane;
        body.pair(dx, dy, dz, r2, pj, j, a);
    }
}

// A full cluster (G = 1): every lane tests the same supplier, read through
// the scalar unit.  Two record sets alternate so that the load of the next
// supplier is in flight while the current one is evaluated.
template <bool SHIFT, class Body>
__device__ __forceinline__ void range_loop_full(Body &body, double xi, double yi, double zi,
                                                int j0, int j1, double shx, double shy,
                                                double shz, const PairArgs &a,
                                                int &n_lane) {
    j0 = __builtin_amdgcn_readfirstlane(j0);
    j1 = __builtin_amdgcn_readfirstlane(j1);
    // the sorted array is padded by kSupplierPad records: the look-ahead
    // loads past j1 stay inside the allocation
    double4 A = load_uniform(a.sp, j0);
    for (int j = j0; j < j1; j += 2) {
        const double4 B = load_uniform(a.sp, j + 1);
        test_pair<SHIFT>(body, xi, yi, zi, A, j, true, shx, shy, shz, a, n_lane);
        A = load_uniform(a.sp, j + 2);
        test_pair<SHIFT>(body, xi, yi, zi, B, j + 1, j + 1 < j1, shx, shy, shz, a, n_lane);
    }
}

// The wave holds G copies ("groups") of the cluster's receivers; group g
// takes suppliers j0 + g, j0 + g + G, ...  Lanes past the last group, and
// groups past the end of the range, test a supplier that cannot pass.
template <bool SHIFT, class Body>
__device__ __forceinline__ void range_loop(Body &body, double xi, double yi, double zi, int j0,
                                           int j1, int grp, int G, double shx, double shy,
                                           double shz, const PairArgs &a,
                                           unsigned long long &n_ok, int &n_lane) {
    if (G == 1) {
        range_loop_full<SHIFT>(body, xi, yi, zi, j0, j1, shx, shy, shz, a, n_lane);
        return;
    }
    const double rc2 = a.g.rc2;
    j0 = __builtin_amdgcn_readfirstlane(j0);
    const int len = __builtin_amdgcn_readfirstlane(j1) - j0;
    // the sorted array is padded by kSupplierPad >= 2*64 records, so the
    // strided reads of the last step and the prefetch after it stay inside
    // the allocation
    const double4 *__restrict__ base = a.sp + j0;
    double4 nxt = base[grp];
    unsigned cnt = 0;
    for (int k = 0; k < len; k += G) {
        const double4 pj = nxt;
        nxt = base[k + G + grp];   // next step's supplier, loaded one step ahead
        const bool ok = grp < len - k;
        double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
        if (SHIFT) {
            dx -= shx;
            dy -= shy;
            dz -= shz;
        }
        const double r2 = dist2(dx, dy, dz);
        cnt += (unsigned)__builtin_popcountll(ballot64(ok) & ballot64(r2 < rc2) &
                                              ballot64(r2 > 0.0));
        if (ok & (r2 < rc2) & (r2 > 0.0)) body.pair(dx, dy, dz, r2, pj, j0 + k + grp, a);
    }
    n_ok += cnt;
}

// Screened suppliers in LDS: group g takes list entries g, g + G, ...; all
// lanes of a group read the same record (an LDS broadcast).  `p` is this
// lane's view of the list (list + min(grp, G)).  The G records after the
// last entry hold far-away points, so a step needs no bounds test; two
// record sets alternate so that the next read is in flight while the
// current record is evaluated.  G is a compile-time constant (64 / csize),
// so the reads use immediate offsets.
template <bool NEED_W>
__device__ __forceinline__ double4 list_read(const double4 *p) {
    if constexpr (NEED_W) {
        return *p;
    } else {
        const double2 xy = *reinterpret_cast<const double2 *>(p);
        return make_double4(xy.x, xy.y, p->z, 0.0);
    }
}

template <bool NEED_W>
__device__ __forceinline__ void list_write(double4 *p, const double4 &v) {
    if constexpr (NEED_W) {
        *p = v;
    } else {
        *reinterpret_cast<double2 *>(p) = make_double2(v.x, v.y);
        p->z = v.z;
    }
}

// One receiver lane against one listed supplier that carries its adjoint
// weight (the weight is unused by the forward bodies).
template <bool SHIFT, class Body>
__device__ __forceinline__ void test_pair_w(Body &body, double xi, double yi, double zi,
                                            const double4 &pj, const typename Body::WT &wj,
                                            double shx, double shy, double shz,
                                            const PairArgs &a, unsigned &n_ok) {
    double dx = xi - pj.x, dy = yi - pj.y, dz = zi - pj.z;
    if (SHIFT) {
        dx -= shx;
        dy -= shy;
        dz -= shz;
    }
    const double r2 = dist2(dx, dy, dz);
    n_ok += count_pass(r2, a.g.rc2);
    if ((r2 < a.g.rc2) & (r2 > 0.0)) body.pair_w(dx, dy, dz, r2, pj, wj, a);
}

// wp: this lane's view of the list's weights (adjoint bodies only).
template <int G, bool SHIFT, class Body>
__device__ __forceinline__ void list_loop(Body &body, const double4 *p,
                                          const typename Body::WT *wp, int n_list, double xi,
                                          double yi, double zi, double shx, double shy,
                                          double shz, const PairArgs &a,
                                          unsigned long long &n_ok) {
    constexpr bool W = Body::kNeedW;
    using WT = typename Body::WT;
    double4 A = list_read<W>(p);
    WT wA{};
    if constexpr (Body::kHasW) wA = wp[0];
    unsigned cnt = 0;
    for (int k = 0; k < n_list; k += 2 * G) {
        const double4 *q = p + k;
        const double4 B = list_read<W>(q + G);
        WT wB{};
        if constexpr (Body::kHasW) wB = wp[k + G];
        test_pair_w<SHIFT>(body, xi, yi, zi, A, wA, shx, shy, shz, a, cnt);
        A = list_read<W>(q + 2 * G);
        if constexpr (Body::kHasW) wA = wp[k + 2 * G];
        if (k + G < n_list)
            test_pair_w<SHIFT>(body, xi, yi, zi, B, wB, shx, shy, shz, a, cnt);
    }
    n_ok += cnt;
}

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Per-wave statistics, kept in registers until the wave runs out of work: a
// contended atomic per item would also delay the next item's loads (vector
// memory operations retire in order).
struct WaveCounts {
    unsigned long long n_ok = 0;        // accepted pairs of the wave (wave-uniform)
    int n_lane = 0;                     // per lane: accepted pairs of the scalar-load loop
    unsigned long long cand = 0;        // receiver x supplier pairs handed to the pair loop
    unsigned long long steps = 0;       // wave steps of the pair loop
    unsigned long long screened = 0;    // supplier records tested against the cluster box
};

// Shared state of one work item for the visitors below.
struct ItemCtx {
    double xi, yi, zi;     // this lane's receiver (far away for idle lanes)
    const double *lo, *hi; // the cluster's bounding box
    int lane, grp, G, cnt;
    int rgrp;              // screened loop: min(grp, G)
};

// Direct visitor: every supplier of every surviving subtile run goes to the
// pair loop.
template <class Body>
struct DirectVisit {
    Body &body;
    const ItemCtx &c;
    const PairArgs &a;
    WaveCounts &wc;
    bool shifted = false;
    double shx = 0.0, shy = 0.0, shz = 0.0;
    __device__ __forceinline__ void tile(int, int, bool sh, double x, double y, double z) {
        shifted = sh;
        shx = x;
        shy = y;
        shz = z;
    }
    __device__ __forceinline__ void run(int j0, int j1) {
        wc.cand += (unsigned long long)(j1 - j0) * (unsigned long long)c.cnt;
        wc.steps += (unsigned long long)((j1 - j0 + c.G - 1) / c.G);
        if (shifted)
            range_loop<true>(body, c.xi, c.yi, c.zi, j0, j1, c.grp, c.G, shx, shy, shz, a, wc.n_ok,
                             wc.n_lane);
        else
            range_loop<false>(body, c.xi, c.yi, c.zi, j0, j1, c.grp, c.G, 0.0, 0.0, 0.0, a,
                              wc.n_ok, wc.n_lane);
    }
    __device__ __forceinline__ void finish() {}
};

// Screening visitor.  Supplier runs are packed into chunks of 64 records
// (one per lane, several runs per chunk, so short runs do not leave lanes
// idle); each full chunk is screened: every lane tests its record against the
// cluster's bounding box (distance from the box below r_cut, conservative by
// the culling margin) and the survivors are appended to the wave's LDS list.
// The list goes to the pair loop when it is nearly full, when the next tile
// has another periodic image, and at the end of the item.  G = 64 / csize
// copies of the cluster share the wave.
template <int G, int CAP, class Body>
struct ScreenVisit {
    static constexpr bool W = Body::kNeedW;
    Body &body;
    const ItemCtx &c;
    const PairArgs &a;
    WaveCounts &wc;
    double4 *list;
    typename Body::WT *wlist;   // adjoint: the listed suppliers' weights (else unused)
    int n_list = 0;
    int code = -1;   // periodic image of the records in the list and the open chunk
    double shx = 0.0, shy = 0.0, shz = 0.0;
    int fill = 0;    // records in the open chunk: lanes [0, fill)
    int jj = 0;      // per lane: its record is a.sp[jj + lane]

    __device__ __forceinline__ void flush() {
        if (n_list == 0) return;
        // far-away records after the last entry: the pair loop's reads past
        // n_list (at most G of them) cannot pass the cut-off
        if (c.lane < 2 * G)
            list_write<W>(list + n_list + c.lane, make_double4(-1.0e300, -1.0e300, -1.0e300, 0.0));
        wave_lds_sync();
        wc.cand += (unsigned long long)n_list * (unsigned long long)c.cnt;
        wc.steps += (unsigned long long)((n_list + G - 1) / G);
        const double4 *p = list + c.rgrp;
        const typename Body::WT *wp = wlist + c.rgrp;
        if (code != 13)
            list_loop<G, true>(body, p, wp, n_list, c.xi, c.yi, c.zi, shx, shy, shz, a, wc.n_ok);
        else
            list_loop<G, false>(body, p, wp, n_list, c.xi, c.yi, c.zi, 0.0, 0.0, 0.0, a,
                                wc.n_ok);
        wave_lds_sync();
        n_list = 0;
    }
    __device__ __forceinline__ double4 load(const double4 *r) const {
        if constexpr (W) {
            return *r;
        } else {
            const double2 xy = *reinterpret_cast<const double2 *>(r);
            return make_double4(xy.x, xy.y, r->z, 0.0);
        }
    }
    // Screen the open chunk.  Lanes past `fill` read a record at most 63
    // past the end of the last run (inside the padded sorted array); they
    // are left out of the count, and what they write lies past the list's
    // last entry.
    __device__ __forceinline__ void screen_chunk() {
        if (fill == 0) return;
        const double4 p = load(a.sp + (jj + c.lane));
        const double px = p.x + shx, py = p.y + shy, pz = p.z + shz;
        const double gx = fmax(0.0, fmax(c.lo[0] - px, px - c.hi[0]));
        const double gy = fmax(0.0, fmax(c.lo[1] - py, py - c.hi[1]));
        const double gz = fmax(0.0, fmax(c.lo[2] - pz, pz - c.hi[2]));
        const bool keep = gx * gx + gy * gy + gz * gz < a.g.cull2;
        const unsigned long long tail = fill >= kWave ? ~0ull : ((1ull << fill) - 1ull);
        const unsigned long long m = ballot64(keep) & tail;
        const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (keep) {
            list_write<W>(list + n_list + off, p);
            // the adjoint's supplier weight (the padded weight array covers
            // the reads of lanes past `fill`)
            if constexpr (Body::kHasW) wlist[n_list + off] = Body::weight(a, jj + c.lane);
        }
        n_list += __builtin_popcountll(m);
        fill = 0;
        if (n_list > CAP - kWave) flush();   // keeps n_list <= CAP
    }
    __device__ __forceinline__ void tile(int, int img, bool, double x, double y, double z) {
        if (img != code) {
            screen_chunk();
            flush();
            code = img;
            shx = x;
            shy = y;
            shz = z;
        }
    }
    __device__ __forceinline__ void run(int j0, int j1) {
        j0 = __builtin_amdgcn_readfirstlane(j0);
        j1 = __builtin_amdgcn_readfirstlane(j1);
        wc.screened += (unsigned long long)(j1 - j0);
        while (j0 < j1) {
            // lanes [fill, fill + take) take records j0, j0 + 1, ...; lanes
            // past them keep the same offset (their reads stay near the run)
            if (c.lane >= fill) jj = j0 - fill;
            const int take = min(j1 - j0, kWave - fill);
            j0 += take;
            fill += take;
            if (fill == kWave) screen_chunk();
        }
    }
    __device__ __forceinline__ void finish() {
        screen_chunk();
        flush();
    }
};

// Floor of (i + 0.5) * inv for 0 <= i < 2^20, inv = 1/d rounded to float, d <= 4096:
// exact, since (i + 0.5) / d is at least 0.5/d away from an integer and the
// float product is off by far less.
__device__ __forceinline__ int div_small(int i, float inv) {
    return (int)(((float)i + 0.5f) * inv);
}

// One work item: the cluster's receivers against the suppliers of its
// neighbour-tile / subtile range.  The item's (tile, subtile) entries are
// tested 64 at a time, one lane each: the subtile box (in the unwrapped
// frame of the tile's periodic image) against the cluster's bounding box,
// the subtile-pair culling of section 2.1.3 done against the receivers'
// actual extent (conservative by the culling margin, so rounding in the box
// corners cannot drop a pair).  Each lane also loads its subtile's cell
// range.  Per neighbour tile of the pass, the image is fixed and consecutive
// surviving subtiles merge into supplier ranges handed to the visitor.
template <class Visit>
__device__ __forceinline__ void walk_item(Visit &v, const Item &item, const Cluster &cl,
                                          const PairArgs &a, int lane) {
    const Geom &g = a.g;
    const int *__restrict__ cs = a.cell_start;
    const double *lo = cl.lo, *hi = cl.hi;
    const int tx = cl.tile / (g.nt * g.nt), ty = (cl.tile / g.nt) % g.nt, tz = cl.tile % g.nt;
    const int t0 = item.tiles & 0xff, t1 = (item.tiles >> 8) & 0xff;
    const int s0 = item.subs & 0xffff, s1 = (item.subs >> 16) & 0xffff;
    const int S = s1 - s0;                 // subtiles of each tile in this item
    const int E = (t1 - t0) * S;           // (tile, subtile) entries
    const int nss = g.ns * g.ns;
    const float inv_S = 1.0f / (float)S;
    const float inv_nss = 1.0f / (float)nss;
    const float inv_ns = 1.0f / (float)g.ns;
    for (int e0 = 0; e0 < E; e0 += kWave) {
        const int e = e0 + lane;
        bool keep = false;
        int cst = 0, cen = 0;
        if (e < E) {
            const int q = div_small(e, inv_S);
            const int s = s0 + e - q * S;
            const int t = t0 + q;
            const int sa = div_small(s, inv_nss);
            const int r = s - sa * nss;
            const int sb = div_small(r, inv_ns);
            const int sc = r - sb * g.ns;
            // unwrapped tile coordinates of the neighbour tile
            const int ux = tx + t / 9 - 1, uy = ty + (t / 3) % 3 - 1, uz = tz + t % 3 - 1;
            const double bx0 = (double)(ux * g.ns + sa) * g.sub;
            const double by0 = (double)(uy * g.ns + sb) * g.sub;
            const double bz0 = (double)(uz * g.ns + sc) * g.sub;
            const double gx = fmax(0.0, fmax(bx0 - hi[0], lo[0] - (bx0 + g.sub)));
            const double gy = fmax(0.0, fmax(by0 - hi[1], lo[1] - (by0 + g.sub)));
            const double gz = fmax(0.0, fmax(bz0 - hi[2], lo[2] - (bz0 + g.sub)));
            keep = gx * gx + gy * gy + gz * gz < g.cull2;
            const int wx = ux < 0 ? ux + g.nt : (ux >= g.nt ? ux - g.nt : ux);
            const int wy = uy < 0 ? uy + g.nt : (uy >= g.nt ? uy - g.nt : uy);
            const int wz = uz < 0 ? uz + g.nt : (uz >= g.nt ? uz - g.nt : uz);
            const int c = ((wx * g.nt + wy) * g.nt + wz) * g.ns3 + s;
            cst = cs[c];
            cen = cs[c + 1];
        }
        const unsigned long long mask = ballot64(keep);
        if (!mask) continue;
        // the neighbour tiles whose entries lie in this pass
        const int e1 = min(E, e0 + kWave);
        for (int q = e0 / S; q * S < e1; ++q) {
            const int la = max(q * S - e0, 0), lb = min((q + 1) * S - e0, kWave);
            const unsigned long long range =
                (lb >= kWave ? ~0ull : ((1ull << lb) - 1ull)) & ~((1ull << la) - 1ull);
            unsigned long long m = mask & range;
            if (!m) continue;
            const int t = t0 + q;
            int nx = tx + t / 9 - 1, ny = ty + (t / 3) % 3 - 1, nz = tz + t % 3 - 1;
            const int ix = nx < 0 ? -1 : (nx >= g.nt ? 1 : 0);
            const int iy = ny < 0 ? -1 : (ny >= g.nt ? 1 : 0);
            const int iz = nz < 0 ? -1 : (nz >= g.nt ? 1 : 0);
            v.tile(t, (ix + 1) * 9 + (iy + 1) * 3 + (iz + 1), (ix | iy | iz) != 0, ix * g.box,
                   iy * g.box, iz * g.box);
            while (m) {
                const int ra = __builtin_ctzll(m);
                const unsigned long long rest = ~(m >> ra);
                const int rb = rest ? ra + __builtin_ctzll(rest) : kWave;   // run [ra, rb)
                const int j0 = __builtin_amdgcn_readlane(cst, ra);
                const int j1 = __builtin_amdgcn_readlane(cen, rb - 1);
                m = rb >= kWave ? 0ull : (m & (~0ull << rb));
                if (j1 > j0) v.run(j0, j1);
            }
        }
    }
    v.finish();
}

// Sum a value over the G copies of each receiver: after the loop, lane
// il (group 0) holds the total of lanes il, il + cnt, ..., il + (G-1) cnt.
__device__ inline double group_sum(double v, int lane, int grp, int cnt, int G) {
    for (int step = 1; step < G; step <<= 1) {
        const double o = __shfl(v, (lane + step * cnt) & (kWave - 1), kWave);
        if ((grp & (2 * step - 1)) == 0 && grp + step < G) v += o;
    }
    return v;
}

// Next work item for this wave.  Items are cut into kXcds contiguous chunks
// (the item list follows the tile order, so a chunk is a compact region of
// the box); the workgroups of XCD x (blockIdx % kXcds, the round-robin
// dispatch order) draw from chunk x through its own counter, so that XCD's
// L2 serves a compact set of suppliers, and steal from the other chunks once
// theirs is empty.  A wave claims a.batch consecutive items per atomic: the
// counters are device-wide, and one atomic per item would serialise on them.
// Returns -1 when every chunk is exhausted.
struct ItemCursor {
    int cur = 0, end = 0;   // claimed items [cur, end)
    int victim = 0;         // chunks tried so far, from the home chunk on
};

// The launch's item count (read on the device) and the items a wave claims
// per queue atomic: about 32 claims per wave, at most 8 items each.
struct ItemQueue {
    int n;
    int batch;
};
__device__ inline ItemQueue item_queue(const PairArgs &a) {
    const int n = __builtin_amdgcn_readfirstlane(*a.n_items_dev);
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    const long long b = (long long)n / (waves * 32);
    return ItemQueue{n, (int)(b < 1 ? 1 : (b > 8 ? 8 : b))};
}

__device__ inline int next_item(const PairArgs &a, const ItemQueue &iq, int lane, ItemCursor &q) {
    if (q.cur < q.end) return q.cur++;
    const int home = (int)(blockIdx.x % kXcds);
    while (q.victim < kXcds) {
        const int x = (home + q.victim) % kXcds;
        const int c0 = (int)((long long)iq.n * x / kXcds);
        const int c1 = (int)((long long)iq.n * (x + 1) / kXcds);
        int got = 0;
        if (lane == 0) got = atomicAdd(a.queue + x * kQueueStride, iq.batch);
        got = __builtin_amdgcn_readfirstlane(got);
        if (c0 + got < c1) {
            q.cur = c0 + got;
            q.end = min(c0 + got + iq.batch, c1);
            return q.cur++;
        }
        ++q.victim;
    }
    return -1;
}

template <int SG, int CAP, class Body>
__device__ __forceinline__ void visit_item(Body &body, const Item &item, const Cluster &cl,
                                           const ItemCtx &c, const PairArgs &a, WaveCounts &wc,
                                           double4 *list, void *wlist) {
    if constexpr (SG > 0) {
        ScreenVisit<SG, CAP, Body> v{body, c, a, wc, list, (typename Body::WT *)wlist};
        walk_item(v, item, cl, a, c.lane);
    } else {
        DirectVisit<Body> v{body, c, a, wc};
        walk_item(v, item, cl, a, c.lane);
    }
}

// Per-supplier adjoint weight kept beside a screened list entry.
template <int MODE> struct ModeWeight { using T = float; };
template <> struct ModeWeight<BWD_F64> { using T = double4; };
template <> struct ModeWeight<BWD_F32> { using T = float4; };

// The persistent pair kernel.  SG > 0 (forward modes only): suppliers are
// screened against the cluster's box into LDS before the pair loop, with SG =
// 64 / csize copies of each cluster per wave; SG = 0: suppliers stream
// directly, with 64 / count copies.  SOFT: B-spline softening inside eps_b.
// Six waves per SIMD for the FP32 forward kernel with unit masses, no
// softening and the polynomial shape: it is limited by issue latency more
// than by VALU throughput and runs about 5 % faster at six waves (80 VGPRs,
// 5 registers spilled outside the pair loop, 26 KB of list LDS per block)
// than at five (2.78 -> 2.64 ms on N = 128^3 clustered).  With per-particle
// masses (19 registers spilled) two runs gave -3 % and +0.7 %; the softened
// kernel (103 VGPRs, four waves) gained nothing at five; the tabulated ones
// are held to fewer waves by the table in LDS; the FP64 ones measured slower
// at six.  Those keep the compiler's choice.  Seven waves (72 VGPRs, 20
// registers spilled) were slower again: 2.79 against 2.68 ms.
template <int MODE, bool UNIT, bool SOFT, int TAB>
struct PairsSix {
    static constexpr bool v = MODE == FWD_F32 && UNIT && !SOFT && TAB == SHAPE_POLY;
};

template <int MODE, bool UNIT, int SG, bool SOFT, int TAB = SHAPE_POLY>
__global__ __launch_bounds__(kForceBlock)
__attribute__((amdgpu_waves_per_eu(PairsSix<MODE, UNIT, SOFT, TAB>::v ? 6 : 1)))
void k_pairs(PairArgs a) {
    constexpr bool SCREEN = SG > 0;
    constexpr bool BWD = MODE == BWD_F32 || MODE == BWD_F64;
    // the adjoint's list entries also carry the supplier's weight: a
    // shorter list keeps the LDS per block at or below 40 KB; the six-wave
    // variant's list fits six blocks per CU
    constexpr int CAP = BWD ? kListCapAdjoint
                            : (PairsSix<MODE, UNIT, SOFT, TAB>::v ? kListCapF32 : kListCap);
    constexpr int NW = kForceBlock / kWave;
    using WTk = typename ModeWeight<MODE>::T;
    __shared__ double4 lists[SCREEN ? NW : 1][SCREEN ? CAP + kListSlack : 1];
    __shared__ WTk wlists[SCREEN && BWD ? NW : 1][SCREEN && BWD ? CAP + kListSlack : 1];
    __shared__ float tabs[TAB != SHAPE_POLY ? kTabFloats : 1];
    if constexpr (TAB != SHAPE_POLY) {
        const int nf = TAB == SHAPE_TAB_LINEAR ? 2 * a.tab_n : a.tab_n;
        for (int k = threadIdx.x; k < nf; k += blockDim.x) tabs[k] = a.htab[k];
        __syncthreads();
    }
    const int lane = threadIdx.x & (kWave - 1);
    double4 *list = lists[SCREEN ? threadIdx.x / kWave : 0];
    void *wlist = wlists[SCREEN && BWD ? threadIdx.x / kWave : 0];
    ItemCursor cursor;
    WaveCounts wc;
    const ItemQueue iq = item_queue(a);
    for (int it = next_item(a, iq, lane, cursor); it >= 0; it = next_item(a, iq, lane, cursor)) {
        const Item item = a.items[it];
        const Cluster cl = a.clusters[item.cluster];
        // receivers replicated over G lane groups; lanes past G*cnt are idle
        ItemCtx c;
        c.cnt = __builtin_amdgcn_readfirstlane(cl.count);
        // the screened loop carries exactly SG copies (count <= csize)
        c.G = SCREEN ? SG : __builtin_amdgcn_readfirstlane(kWave / c.cnt);
        c.lane = lane;
        c.grp = lane / c.cnt;
        c.rgrp = min(c.grp, c.G);
        c.lo = cl.lo;
        c.hi = cl.hi;
        const int il = lane - c.grp * c.cnt;
        const bool live = c.grp < c.G;
        const double4 xp = a.rp[cl.begin + il];
        // idle lanes sit far outside the box: no pair passes r < r_cut
        const double far = live ? 0.0 : 1.0e300;
        c.xi = xp.x + far;
        c.yi = xp.y + far;
        c.zi = xp.z + far;
        double ax, ay, az;
        if constexpr (MODE == FWD_F32) {
            FwdF32<UNIT, SOFT, TAB> b;
            b.tab = tabs;
            visit_item<SG, CAP>(b, item, cl, c, a, wc, list, wlist);
            ax = b.ax; ay = b.ay; az = b.az;
        } else if constexpr (MODE == FWD_F64) {
            FwdF64<UNIT, SOFT> b;
            visit_item<SG, CAP>(b, item, cl, c, a, wc, list, wlist);
            ax = b.ax; ay = b.ay; az = b.az;
        } else if constexpr (MODE == BWD_F64) {
            BwdF64<SOFT> b;
            const double4 w = a.rwa[cl.begin + il];
            b.wkx = w.x; b.wky = w.y; b.wkz = w.z; b.muk = xp.w;
            visit_item<SG, CAP>(b, item, cl, c, a, wc, list, wlist);
            ax = b.ax; ay = b.ay; az = b.az;
        } else {
            BwdF32<SOFT> b;
            const float4 w = reinterpret_cast<const float4 *>(a.rwa)[cl.begin + il];
            b.wkx = w.x; b.wky = w.y; b.wkz = w.z; b.muk = mu_f32(xp.w);
            visit_item<SG, CAP>(b, item, cl, c, a, wc, list, wlist);
            ax = b.ax; ay = b.ay; az = b.az;
        }
        if (c.G > 1) {
            ax = group_sum(ax, lane, c.grp, c.cnt, c.G);
            ay = group_sum(ay, lane, c.grp, c.cnt, c.G);
            az = group_sum(az, lane, c.grp, c.cnt, c.G);
        }
        // group 0 holds the item's sums: stored when the item is its
        // cluster's only one, else added (FP64 atomics) into the zeroed output,
        // or, in the deterministic mode, stored in the item's partial slot
        // for the ordered reduction after the launch
        if (c.grp == 0) {
            double *o = a.out + (long long)cl.subset * a.out_stride + 3ll * a.rperm[cl.begin + il];
            if (item.sole & kItemSole) {
                o[0] = ax;
                o[1] = ay;
                o[2] = az;
            } else if (a.partials) {
                double *q = a.partials + ((size_t)it * a.csize + il) * 3;
                q[0] = ax;
                q[1] = ay;
                q[2] = az;
            } else {
                atomicAdd(o, ax);
                atomicAdd(o + 1, ay);
                atomicAdd(o + 2, az);
            }
        }
    }
    unsigned long long tot = (unsigned long long)wc.n_lane;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off, kWave);
    tot += wc.n_ok;
    if (lane == 0 && a.counters && wc.steps + wc.screened + wc.cand + tot > 0) {
        Counters *k = a.counters + (blockIdx.x % kCounterCopies) * kCounterStride;
        atomicAdd(&k->interactions, tot);
        atomicAdd(&k->candidates, wc.cand);
        atomicAdd(&k->steps, wc.steps);
        atomicAdd(&k->screened, wc.screened);
    }
}

// ---- pairs evaluated once for both partners -----------------------------------
//
// All-active FP32 forward calls: each unordered pair {i, j} is evaluated once
// and its force is applied to both particles (Newton's third law; the
// receiver/supplier tile pairing of section 2.1.3, "Tiles", visits each tile
// pair once for the same reason).  A cluster visits only the upper half of
// its 27-tile stencil (t = 13 .. 26, whose mirror images are the lower half)
// and, in its own tile, only the particles after it; its own pairs are
// evaluated separately (below).
//
// Lanes form four rows of 16.  A cluster of 16 R receivers (R = 1, 2, 4) sits
// in the rows with receiver 16 (row % R) + lane; the screened suppliers come
// in blocks of 16 (4 / R) list entries, row r holding entries 16 (r / R) ..
// + 15, so the R rows that share a block hold the cluster's R parts.  In 16
// steps each lane meets every entry of its row: at step S it takes the entry
// S places along its row (a DPP row rotation, folded into the subtraction
// that forms the separation), and the reaction goes back to the entry's own
// lane by the opposite rotation (folded into the addition).  After the block
// the R rows' reactions on an entry are summed and added to the supplier's
// total with one FP64 atomic per component.
//
// Precision (FP32 on cluster-relative coordinates; positions, the periodic
// image and the sums stay FP64): every particle enters the block as its
// offset from the centre of the cluster's box, rounded to FP32 (suppliers
// with their periodic image applied in FP64 first).  The separation, r^2
// and the cut-off test are FP32.  Two rare cases take the FP64 positions
// instead, so that the accepted pairs are exactly those of the plain FP64
// evaluation and close pairs keep FP32 relative accuracy:
//   - r^2 within a relative 2^-17 of r_cut^2 (the FP32 r^2 is within 2^-20
//     of the exact one for offsets up to 2.2 r_cut, the largest a cluster
//     inside one tile can have): the test is repeated in FP64;
//   - r below a tenth of the receiver's offset, where the rounding of the
//     offsets (2^-24 of their size) would exceed 2^-21 of r: the separation
//     is recomputed in FP64 and rounded.
// The pair factor is the FP32 shape of FwdF32 (hardware rsqrt and the H
// polynomial); a block's sums are FP32 over its 16 steps and then FP64.
//
// The FP64 kinds (forward, softened forward and adjoint of FP64 calls) keep
// the offsets, the pair term and every sum in FP64; a rotated FP64 operand
// takes two DPP moves, and the two rare cases are a relative 2^-40 band
// around r_cut^2 and the same close-pair rule, redone in the plain form
// (x_i - x_j) - n' box.
//
// The sums go to an FP64 array in sorted order, one component after the
// other (three arrays of n), which a final pass writes to acc_out.

// The mutual kernels' call kinds: the forward force, the adjoint, the
// forward force with B-spline softening.
constexpr int kMutFwd = 0, kMutBwd = 1, kMutSoft = 2;
// The FP64 forward force, the FP64 adjoint and the softened FP64 forward
// force: FP64 offsets, separations, pair terms and sums.
constexpr int kMutF64 = 3, kMutF64Bwd = 4, kMutF64Soft = 5;
template <int KIND>
constexpr bool kMutIsF64 = KIND == kMutF64 || KIND == kMutF64Bwd || KIND == kMutF64Soft;
template <int KIND> constexpr bool kMutIsBwd = KIND == kMutBwd || KIND == kMutF64Bwd;

template <bool B, class T, class F> struct MutPick { using type = T; };
template <class T, class F> struct MutPick<false, T, F> { using type = F; };
// A list entry in the ring (offset from the cluster centre and mu), and an
// entry's adjoint weight: FP32, or FP64 for the FP64 kinds.
template <int KIND> using MutEntry = typename MutPick<kMutIsF64<KIND>, double4, float4>::type;

constexpr int kRing = 128;                    // list entries per wave (a ring)
constexpr unsigned kIdxBits = 27;             // sorted index bits of a list entry
constexpr unsigned kIdxMask = (1u << kIdxBits) - 1u;

// The value of the lane S places along this lane's row of 16 (DPP row
// rotation; every source lane is valid, so the move can fold into the VALU
// instruction that uses it).
template <int S>
__device__ __forceinline__ float rot16(float v) {
    if constexpr (S == 0) {
        return v;
    } else {
        return __builtin_bit_cast(
            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + S, 0xf, 0xf, true));
    }
}
template <int S>
__device__ __forceinline__ int rot16i(int v) {
    if constexpr (S == 0) return v;
    else return __builtin_amdgcn_mov_dpp(v, 0x120 + S, 0xf, 0xf, true);
}
// An FP64 value: two DPP moves (a rotation does not fold into FP64
// instructions).
template <int S>
__device__ __forceinline__ double rot16(double v) {
    if constexpr (S == 0) {
        return v;
    } else {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)rot16i<S>((int)(unsigned)b);
        const unsigned hi = (unsigned)rot16i<S>((int)(unsigned)(b >> 32));
        return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
    }
}

// v where this lane's bit of the wave mask is set, else 0: one v_cndmask
// with the mask as its selector.
__device__ __forceinline__ float keep_lanes(unsigned long long mask, float v) {
    float r;
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(r) : "v"(v), "s"(mask));
    return r;
}

// v where this lane's bit of the wave mask is set, else 0 (FP64: both halves).
__device__ __forceinline__ double keep_lanes(unsigned long long mask, double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    unsigned lo, hi;
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(lo) : "v"((unsigned)b), "s"(mask));
    asm("v_cndmask_b32 %0, 0, %1, %2" : "=v"(hi) : "v"((unsigned)(b >> 32)), "s"(mask));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// This lane's receiver and its sums.
struct MutualLane {
    float hx, hy, hz;     // offset from the cluster centre (far away for idle lanes)
    float ki;             // r^2 below which the separation is recomputed in FP64
    float mu;             // mu_i (FP32)
    int i_sorted;
    float axf = 0.f, ayf = 0.f, azf = 0.f;   // block sums (FP32)
    float jx = 0.f, jy = 0.f, jz = 0.f;      // reaction on this lane's entry (FP32)
    float wkx = 0.f, wky = 0.f, wkz = 0.f;   // adjoint: this receiver's w_k [k active]
    float eb2 = 0.f;                         // softened forward: eps_b^2 (FP32)
};

// The separation of receiver i_sorted and list entry jr (sorted index |
// image << kIdxBits) from the FP64 positions, as the plain evaluation forms
// it: (x_i - x_j) - n' box, rounded to FP32 with its r^2 (w < 0: the pair
// fails 0 < r^2 < r_cut^2).  Out of line: it runs for about one step in a
// thousand.
__device__ __attribute__((noinline)) float4 mutual_fp64_sep(const double4 *__restrict__ sp,
                                                            int i_sorted, int jr, double box,
                                                            double rc2) {
    const int j = (int)((unsigned)jr & kIdxMask);
    const int img = (int)((unsigned)jr >> kIdxBits);
    const double4 pi = sp[i_sorted];
    const double4 pj = sp[j];
    double ddx = pi.x - pj.x, ddy = pi.y - pj.y, ddz = pi.z - pj.z;
    if (img != 13) {
        ddx -= (double)(img / 9 - 1) * box;
        ddy -= (double)((img / 3) % 3 - 1) * box;
        ddz -= (double)(img % 3 - 1) * box;
    }
    const double r2d = dist2(ddx, ddy, ddz);
    const bool ok = (r2d < rc2) & (r2d > 0.0);
    return make_float4((float)ddx, (float)ddy, (float)ddz, ok ? (float)r2d : -1.0f);
}

// One step of a block: this lane's receiver against the entry S places along
// its row.  SELF: the cluster's own particles, each ordered pair evaluated
// from both ends, no reaction.  BWD: the adjoint's pair term instead of the
// force; ew holds the entry's weight w_j [j active].
template <int S, bool UNIT, bool SELF, int KIND>
__device__ __forceinline__ void mutual_step(MutualLane &m, const float4 &e, const float4 &ew,
                                            int jid, const PairArgs &a, unsigned &cnt,
                                            unsigned &rare_n) {
    constexpr bool BWD = KIND == kMutBwd;
    // each step's values die within it: keep the scheduler from interleaving
    // the unrolled steps (which multiplies the live registers)
    __builtin_amdgcn_sched_barrier(0);
    float dx = m.hx - rot16<S>(e.x);
    float dy = m.hy - rot16<S>(e.y);
    float dz = m.hz - rot16<S>(e.z);
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    // pairs decided in FP32: ki <= r^2 < rc2_lo; in FP64: r^2 < ki, and
    // rc2_lo <= r^2 < rc2_hi (the masks are wave-wide, the logic scalar)
    const unsigned long long m_lo = ballot64(r2 < a.rc2_lo);
    const unsigned long long m_far = ballot64(r2 >= m.ki);
    const unsigned long long m_hi = ballot64(r2 < a.rc2_hi);
    unsigned long long acc_m = m_lo & m_far;
    const unsigned long long rare = (m_hi & ~m_lo) | ~m_far;
    if (rare) {
        const int jr = rot16i<S>(jid);   // all lanes active here
        ++rare_n;
        bool ok = false;
        if ((rare >> (threadIdx.x & (kWave - 1))) & 1ull) {
            const float4 q = mutual_fp64_sep(a.sp, m.i_sorted, jr, a.g.box, a.g.rc2);
            ok = q.w > 0.0f;
            dx = q.x;
            dy = q.y;
            dz = q.z;
            r2 = ok ? q.w : 1.0f;
        }
        acc_m = (acc_m & ~rare) | (ballot64(ok) & rare);
    }
    cnt += (unsigned)__builtin_popcountll(acc_m);
    if constexpr (BWD) {
        // the adjoint's term of the pair: receiver k gets -J(r) v and the
        // entry j gets +J(r) v, v = mu_j w_k - mu_k w_j and J(r) v =
        // phi v - c (r . v) r (J is even in r, so the pair term is
        // antisymmetric and each pair is evaluated once for both)
        float vx, vy, vz;
        if constexpr (UNIT) {
            vx = m.wkx - rot16<S>(ew.x);
            vy = m.wky - rot16<S>(ew.y);
            vz = m.wkz - rot16<S>(ew.z);
        } else {
            const float muj = rot16<S>(e.w);
            vx = fmaf(muj, m.wkx, -(m.mu * rot16<S>(ew.x)));
            vy = fmaf(muj, m.wky, -(m.mu * rot16<S>(ew.y)));
            vz = fmaf(muj, m.wkz, -(m.mu * rot16<S>(ew.z)));
        }
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri2 = ri * ri;
        const float ex = __builtin_amdgcn_exp2f(r2 * (float)a.g.k2);
        const float gu = ex * q_poly(fmaf(r2 * ri, a.g.k1f, -P3M_GPOLY_C0));
        const float phi0 = gu * ri2 * ri;   // g / r^3
        // lanes without a pair give no term
        const float phi = keep_lanes(acc_m, phi0);
        const float c = keep_lanes(acc_m, ri2 * fmaf(3.0f, phi0, a.g.kbf * ex));
        const float crv = c * fmaf(dz, vz, fmaf(dy, vy, dx * vx));
        const float ox = fmaf(-crv, dx, phi * vx);
        const float oy = fmaf(-crv, dy, phi * vy);
        const float oz = fmaf(-crv, dz, phi * vz);
        m.axf -= ox;
        m.ayf -= oy;
        m.azf -= oz;
        if constexpr (!SELF) {
            m.jx += rot16<(16 - S) & 15>(ox);
            m.jy += rot16<(16 - S) & 15>(oy);
            m.jz += rot16<(16 - S) & 15>(oz);
        }
        asm volatile("" ::"v"(m.axf), "v"(m.ayf), "v"(m.azf), "v"(m.jx), "v"(m.jy), "v"(m.jz));
        return;
    }
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float h = h_poly(fmaf(r2, a.g.c2f, -P3M_HPOLY_T0));
    const float ri3 = ri * ri * ri;
    float shv = fmaf(a.g.c3f, h, ri3);
    if constexpr (KIND == kMutSoft) {
        // pairs inside the softening length (few): c3 H(t) + |r|_B^-3 with
        // the softening term in FP64, as in the ordered kernel (the factor
        // is continuous at eps_b, so the FP32 test there is enough)
        const unsigned long long m_soft = ballot64(r2 < m.eb2) & acc_m;
        if (m_soft) {
            if ((m_soft >> (threadIdx.x & (kWave - 1))) & 1ull) {
                const double x = (double)(r2 * ri * a.g.inv_eps_bf);
                shv = (float)((double)(a.g.c3f * h) + bspline_m3(x, (double)ri3, a.g));
            }
        }
    }
    // lanes without a pair send no reaction
    const float sh = keep_lanes(acc_m, shv);
    float shj = sh, shi = sh;
    if constexpr (!UNIT) {
        shj = sh * rot16<S>(e.w);          // the force on i carries mu_j
        shi = sh * m.mu;                   // the reaction on j carries mu_i
    }
    // the reaction's products first: a DPP read of a value written by the
    // previous instruction would need wait states
    const float fx = shi * dx, fy = shi * dy, fz = shi * dz;
    m.axf = fmaf(-shj, dx, m.axf);
    m.ayf = fmaf(-shj, dy, m.ayf);
    m.azf = fmaf(-shj, dz, m.azf);
    if constexpr (!SELF) {
        m.jx += rot16<(16 - S) & 15>(fx);
        m.jy += rot16<(16 - S) & 15>(fy);
        m.jz += rot16<(16 - S) & 15>(fz);
    }
    // the sums are formed within the step: left to itself the compiler sinks
    // the chains past the later steps' branches and keeps every step's
    // separation and pair factor alive until the end of the block
    asm volatile("" ::"v"(m.axf), "v"(m.ayf), "v"(m.azf), "v"(m.jx), "v"(m.jy), "v"(m.jz));
}

template <bool UNIT, bool SELF, int NS, int KIND>
__device__ __forceinline__ void mutual_steps(MutualLane &m, const float4 &e, const float4 &ew,
                                             int jid, const PairArgs &a, unsigned &cnt,
                                             unsigned &rare_n) {
    mutual_step<0, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
    mutual_step<1, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
    mutual_step<2, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
    mutual_step<3, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
    if constexpr (NS > 4) {
        mutual_step<4, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<5, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<6, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<7, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<8, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<9, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<10, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<11, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<12, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<13, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<14, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step<15, UNIT, SELF, KIND>(m, e, ew, jid, a, cnt, rare_n);
    }
}

// The FP64 kind: this lane's receiver, its sums (FP64 throughout) and the
// cut-off band (wave-uniform).
struct MutualLane64 {
    double hx, hy, hz;    // offset from the cluster centre (far away for idle lanes)
    double ki;            // r^2 below which the separation is recomputed as the plain form
    double mu;            // mu_i
    double rlo, rhi;      // r_cut^2 (1 -+ 2^-40)
    int i_sorted;
    double ax = 0.0, ay = 0.0, az = 0.0;   // the receiver's sums
    double jx = 0.0, jy = 0.0, jz = 0.0;   // reaction on this lane's entry
    double wkx = 0.0, wky = 0.0, wkz = 0.0;   // adjoint: this receiver's w_k [k active]
};

// mutual_fp64_sep without the rounding to FP32.
__device__ __attribute__((noinline)) double4 mutual_sep_plain(const double4 *__restrict__ sp,
                                                              int i_sorted, int jr, double box,
                                                              double rc2) {
    const int j = (int)((unsigned)jr & kIdxMask);
    const int img = (int)((unsigned)jr >> kIdxBits);
    const double4 pi = sp[i_sorted];
    const double4 pj = sp[j];
    double ddx = pi.x - pj.x, ddy = pi.y - pj.y, ddz = pi.z - pj.z;
    if (img != 13) {
        ddx -= (double)(img / 9 - 1) * box;
        ddy -= (double)((img / 3) % 3 - 1) * box;
        ddz -= (double)(img % 3 - 1) * box;
    }
    const double r2d = dist2(ddx, ddy, ddz);
    const bool ok = (r2d < rc2) & (r2d > 0.0);
    return make_double4(ddx, ddy, ddz, ok ? r2d : -1.0);
}

// One FP64 step: this lane's receiver against the entry S places along its
// row.  The separation of two offsets from the cluster centre can differ
// from the plain form (x_i - x_j) - n' box in its last bits, so pairs within
// a relative 2^-40 of r_cut^2 and pairs closer than a tenth of the
// receiver's offset are redone in the plain form: the accepted pairs are the
// plain form's.
template <int S, bool UNIT, bool SELF, bool BWD, bool SOFT>
__device__ __forceinline__ void mutual_step64(MutualLane64 &m, const double4 &e,
                                              const double4 &ew, int jid, const PairArgs &a,
                                              unsigned &cnt, unsigned &rare_n) {
    __builtin_amdgcn_sched_barrier(0);
    double dx = m.hx - rot16<S>(e.x);
    double dy = m.hy - rot16<S>(e.y);
    double dz = m.hz - rot16<S>(e.z);
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const unsigned long long m_lo = ballot64(r2 < m.rlo);
    const unsigned long long m_far = ballot64(r2 >= m.ki);
    const unsigned long long m_hi = ballot64(r2 < m.rhi);
    unsigned long long acc_m = m_lo & m_far;
    const unsigned long long rare = (m_hi & ~m_lo) | ~m_far;
    if (rare) {
        const int jr = rot16i<S>(jid);   // all lanes active here
        ++rare_n;
        bool ok = false;
        if ((rare >> (threadIdx.x & (kWave - 1))) & 1ull) {
            const double4 q = mutual_sep_plain(a.sp, m.i_sorted, jr, a.g.box, a.g.rc2);
            ok = q.w > 0.0;
            dx = q.x;
            dy = q.y;
            dz = q.z;
            r2 = ok ? q.w : 1.0;
        }
        acc_m = (acc_m & ~rare) | (ballot64(ok) & rare);
    }
    cnt += (unsigned)__builtin_popcountll(acc_m);
    if constexpr (BWD) {
        // the adjoint's term, as in the FP32 kind: receiver k gets -J(r) v
        // and the entry j gets +J(r) v, v = mu_j w_k - mu_k w_j, J(r) v =
        // phi v - c (r . v) r with phi and c of the FP64 screened kernel
        double vx, vy, vz;
        if constexpr (UNIT) {
            vx = m.wkx - rot16<S>(ew.x);
            vy = m.wky - rot16<S>(ew.y);
            vz = m.wkz - rot16<S>(ew.z);
        } else {
            const double muj = rot16<S>(e.w);
            vx = fma(muj, m.wkx, -(m.mu * rot16<S>(ew.x)));
            vy = fma(muj, m.wky, -(m.mu * rot16<S>(ew.y)));
            vz = fma(muj, m.wkz, -(m.mu * rot16<S>(ew.z)));
        }
        const double ri = rsqrt_pos(r2);
        const double ri2 = ri * ri;
        double dh;
        const double h = h64_d(fma(r2, a.g.c2, -P3M_H64_T0), a.g.h64, dh);
        // lanes without a pair give no term
        const double phi = keep_lanes(acc_m, fma(a.g.c3, h, ri2 * ri));
        const double c =
            keep_lanes(acc_m, fma(3.0 * ri2 * ri2, ri, -2.0 * a.g.c2 * a.g.c3 * dh));
        const double crv = c * fma(dz, vz, fma(dy, vy, dx * vx));
        const double ox = fma(-crv, dx, phi * vx);
        const double oy = fma(-crv, dy, phi * vy);
        const double oz = fma(-crv, dz, phi * vz);
        m.ax -= ox;
        m.ay -= oy;
        m.az -= oz;
        if constexpr (!SELF) {
            m.jx += rot16<(16 - S) & 15>(ox);
            m.jy += rot16<(16 - S) & 15>(oy);
            m.jz += rot16<(16 - S) & 15>(oz);
        }
        asm volatile("" ::"v"(m.ax), "v"(m.ay), "v"(m.az), "v"(m.jx), "v"(m.jy), "v"(m.jz));
        return;
    }
    const double ri = rsqrt_pos(r2);
    const double h = h64(fma(r2, a.g.c2, -P3M_H64_T0), a.g.h64);
    const double ri3 = ri * ri * ri;
    double shv = fma(a.g.c3, h, ri3);
    if constexpr (SOFT) {
        // pairs inside the softening length (few): c3 H(t) + |r|_B^-3, as
        // in the screened FP64 kernel
        const unsigned long long m_soft = ballot64(r2 < a.g.eps_b2) & acc_m;
        if (m_soft) {
            if ((m_soft >> (threadIdx.x & (kWave - 1))) & 1ull)
                shv = fma(a.g.c3, h, bspline_m3(r2 * ri * a.g.inv_eps_b, ri3, a.g));
        }
    }
    // lanes without a pair send no reaction
    const double sh = keep_lanes(acc_m, shv);
    double shj = sh, shi = sh;
    if constexpr (!UNIT) {
        shj = sh * rot16<S>(e.w);
        shi = sh * m.mu;
    }
    const double fx = shi * dx, fy = shi * dy, fz = shi * dz;
    m.ax = fma(-shj, dx, m.ax);
    m.ay = fma(-shj, dy, m.ay);
    m.az = fma(-shj, dz, m.az);
    if constexpr (!SELF) {
        m.jx += rot16<(16 - S) & 15>(fx);
        m.jy += rot16<(16 - S) & 15>(fy);
        m.jz += rot16<(16 - S) & 15>(fz);
    }
    asm volatile("" ::"v"(m.ax), "v"(m.ay), "v"(m.az), "v"(m.jx), "v"(m.jy), "v"(m.jz));
}

template <bool UNIT, bool SELF, int NS, bool BWD, bool SOFT>
__device__ __forceinline__ void mutual_steps64(MutualLane64 &m, const double4 &e,
                                               const double4 &ew, int jid, const PairArgs &a,
                                               unsigned &cnt, unsigned &rare_n) {
    mutual_step64<0, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
    mutual_step64<1, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
    mutual_step64<2, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
    mutual_step64<3, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
    if constexpr (NS > 4) {
        mutual_step64<4, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<5, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<6, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<7, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<8, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<9, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<10, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<11, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<12, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<13, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<14, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
        mutual_step64<15, UNIT, SELF, BWD, SOFT>(m, e, ew, jid, a, cnt, rare_n);
    }
}

// Sums over the lanes of the R rows that hold the same block entries
// (rows r and r ^ 1, r ^ 2 for R = 2, 4).
template <int R, class T>
__device__ __forceinline__ T rows_sum(T v) {
    if constexpr (R >= 2) v += __shfl_xor(v, 16, kWave);
    if constexpr (R >= 4) v += __shfl_xor(v, 32, kWave);
    return v;
}

template <int R, bool UNIT, int KIND>
struct MutualVisit {
    static constexpr bool BWD = kMutIsBwd<KIND>;
    static constexpr bool F64 = kMutIsF64<KIND>;
    using Lane = typename MutPick<F64, MutualLane64, MutualLane>::type;
    static constexpr int EB = 64 / R;   // list entries per block of 16 steps
    const PairArgs &a;
    Lane &m;
    MutEntry<KIND> *lpos;   // ring: offset from the cluster centre, mu
    int *lidx;           // ring: sorted index | image << kIdxBits
    MutEntry<KIND> *lw;   // ring (adjoint): the entry's weight w_j [j active]
    const double *lo, *hi;
    double cx, cy, cz;   // the cluster centre
    int lane;
    int own_from;        // own tile: suppliers from this sorted index on
    double ax = 0.0, ay = 0.0, az = 0.0;
    unsigned long long pairs = 0, steps = 0, screened = 0, rare = 0;
    bool own = false;
    int code = 13;
    double shx = 0.0, shy = 0.0, shz = 0.0;
    int fill = 0, jj = 0, head = 0, n_list = 0;

    // FP32 block sums into the FP64 ones (the FP64 kind sums in FP64 throughout)
    __device__ __forceinline__ void flush_i() {
        if constexpr (!F64) {
            ax += (double)m.axf;
            ay += (double)m.ayf;
            az += (double)m.azf;
            m.axf = m.ayf = m.azf = 0.f;
        }
    }
    // an entry's adjoint weight (FP32 records for the FP32 adjoint)
    __device__ __forceinline__ static MutEntry<KIND> wa_entry_of(const PairArgs &a, int j) {
        if constexpr (F64) return a.wa[j];
        else return reinterpret_cast<const float4 *>(a.wa)[j];
    }
    __device__ __forceinline__ MutEntry<KIND> wa_entry(int j) const { return wa_entry_of(a, j); }
    __device__ __forceinline__ static MutEntry<KIND> far_entry() {
        if constexpr (F64) return make_double4(-1.0e30, -1.0e30, -1.0e30, 0.0);
        else return make_float4(-1.0e30f, -1.0e30f, -1.0e30f, 0.f);
    }

    // One block of nv (<= EB) list entries from the ring head.
    __device__ __forceinline__ void block(int nv) {
        wave_lds_sync();
        const int row = lane >> 4;
        const int k = (row / R) * 16 + (lane & 15);
        MutEntry<KIND> e = far_entry();
        MutEntry<KIND> ew{};
        int jid = -1;
        if (k < nv) {
            const int q = (head + k) & (kRing - 1);
            e = lpos[q];
            jid = lidx[q];
            if constexpr (BWD) ew = lw[q];
        }
        wave_lds_sync();   // the reads are done before later screens overwrite the ring
        m.jx = m.jy = m.jz = 0.f;
        unsigned cnt = 0, rn = 0;
        if constexpr (F64)
            mutual_steps64<UNIT, false, 16, BWD, KIND == kMutF64Soft>(m, e, ew, jid, a, cnt, rn);
        else mutual_steps<UNIT, false, 16, KIND>(m, e, ew, jid, a, cnt, rn);
        flush_i();
        const auto jx = rows_sum<R>(m.jx), jy = rows_sum<R>(m.jy), jz = rows_sum<R>(m.jz);
        if (row % R == 0 && k < nv) {
            const int j = (int)((unsigned)jid & kIdxMask);
            atomicAdd(a.out + j, (double)jx);
            atomicAdd(a.out + a.out_stride + j, (double)jy);
            atomicAdd(a.out + 2 * a.out_stride + j, (double)jz);
        }
        pairs += 2ull * cnt;
        steps += 16;
        rare += rn;
    }

    // The cluster's own pairs (cnt <= 16 R particles), from both ends.
    __device__ __forceinline__ void self_pass(int cnt, int begin) {
        const int row = lane >> 4, l = lane & 15;
        constexpr int passes = R == 4 ? 4 : 1;
#pragma unroll 1
        for (int p = 0; p < passes; ++p) {
            // R = 1: row r holds the particles rotated by 4 r, so four steps
            // cover every offset; R = 2: rows 0, 1 meet particles 0..15, rows
            // 2, 3 particles 16..31; R = 4: row r meets part (r + p) % 4.
            int idx;
            if constexpr (R == 1) idx = (l + 4 * row) & 15;
            else if constexpr (R == 2) idx = 16 * (row >> 1) + l;
            else idx = 16 * ((row + p) & 3) + l;
            MutEntry<KIND> e = far_entry();
            MutEntry<KIND> ew{};
            int jid = -1;
            if (idx < cnt) {
                const double4 q = a.sp[begin + idx];
                if constexpr (F64)
                    e = make_double4(q.x - cx, q.y - cy, q.z - cz, UNIT ? 0.0 : q.w);
                else
                    e = make_float4((float)(q.x - cx), (float)(q.y - cy), (float)(q.z - cz),
                                    UNIT ? 0.f : mu_f32(q.w));
                jid = (begin + idx) | (13 << kIdxBits);
                if constexpr (BWD) ew = wa_entry(begin + idx);
            }
            unsigned c = 0, rn = 0;
            if constexpr (F64)
                mutual_steps64<UNIT, true, R == 1 ? 4 : 16, BWD, KIND == kMutF64Soft>(m, e, ew,
                                                                                    jid, a, c, rn);
            else mutual_steps<UNIT, true, R == 1 ? 4 : 16, KIND>(m, e, ew, jid, a, c, rn);
            flush_i();
            pairs += c;
            steps += R == 1 ? 4 : 16;
            rare += rn;
        }
    }

    __device__ __forceinline__ void screen_chunk() {
        if (fill == 0) return;
        // lanes past `fill` read a record at most 63 past the end of the last
        // run, inside the padded sorted array, and keep nothing
        const double4 p = load_rec(a.sp + (jj + lane));
        const double px = p.x + shx, py = p.y + shy, pz = p.z + shz;
        const double gx = fmax(0.0, fmax(lo[0] - px, px - hi[0]));
        const double gy = fmax(0.0, fmax(lo[1] - py, py - hi[1]));
        const double gz = fmax(0.0, fmax(lo[2] - pz, pz - hi[2]));
        const bool keep = (gx * gx + gy * gy + gz * gz < a.g.cull2) & (lane < fill);
        const unsigned long long mk = ballot64(keep);
        const int off = __builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
        if (keep) {
            const int q = (head + n_list + off) & (kRing - 1);
            if constexpr (F64)
                lpos[q] = make_double4(px - cx, py - cy, pz - cz, UNIT ? 0.0 : p.w);
            else
                lpos[q] = make_float4((float)(px - cx), (float)(py - cy), (float)(pz - cz),
                                      UNIT ? 0.f : mu_f32(p.w));
            lidx[q] = (jj + lane) | (code << kIdxBits);
            if constexpr (BWD) lw[q] = wa_entry(jj + lane);
        }
        n_list += __builtin_popcountll(mk);
        fill = 0;
        // n_list < EB before the chunk, so the ring never holds more than
        // EB + 63 <= kRing - 1 entries
        while (n_list >= EB) {
            block(EB);
            head = (head + EB) & (kRing - 1);
            n_list -= EB;
        }
    }
    __device__ __forceinline__ static double4 load_rec(const double4 *r) {
        if constexpr (UNIT) {
            const double2 xy = *reinterpret_cast<const double2 *>(r);
            return make_double4(xy.x, xy.y, r->z, 0.0);
        } else {
            return *r;
        }
    }
    __device__ __forceinline__ void tile(int t, int img, bool, double x, double y, double z) {
        own = t == 13;
        if (img != code) {
            screen_chunk();   // the open chunk was loaded with the previous image
            code = img;
            shx = x;
            shy = y;
            shz = z;
        }
    }
    __device__ __forceinline__ void run(int j0, int j1) {
        j0 = __builtin_amdgcn_readfirstlane(j0);
        j1 = __builtin_amdgcn_readfirstlane(j1);
        if (own) j0 = max(j0, own_from);
        if (j0 >= j1) return;
        screened += (unsigned long long)(j1 - j0);
        while (j0 < j1) {
            if (lane >= fill) jj = j0 - fill;
            const int take = min(j1 - j0, kWave - fill);
            j0 += take;
            fill += take;
            if (fill == kWave) screen_chunk();
        }
    }
    __device__ __forceinline__ void finish() {
        screen_chunk();
        if (n_list > 0) {
            block(n_list);
            head = (head + n_list) & (kRing - 1);
            n_list = 0;
        }
    }
};

// Tallies of a wave's items.
struct MutualTally {
    unsigned long long pairs = 0, steps = 0, screened = 0, rare = 0;
};

// One work item in the layout of R rows per receiver copy (cnt <= 16 R).
template <int R, bool UNIT, int KIND>
__device__ __forceinline__ void mutual_item(const PairArgs &a, const Item &item,
                                            const Cluster &cl, int cnt, int begin, int lane,
                                            MutEntry<KIND> *ring_pos, int *ring_idx,
                                            MutEntry<KIND> *ring_w, MutualTally &tally) {
    constexpr bool BWD = kMutIsBwd<KIND>;
    constexpr bool F64 = kMutIsF64<KIND>;
    const int row = lane >> 4, l = lane & 15;
    const double cx = 0.5 * (cl.lo[0] + cl.hi[0]);
    const double cy = 0.5 * (cl.lo[1] + cl.hi[1]);
    const double cz = 0.5 * (cl.lo[2] + cl.hi[2]);
    typename MutualVisit<R, UNIT, KIND>::Lane m;
    const int idx = 16 * (row % R) + l;
    const bool live = idx < cnt;
    m.i_sorted = begin + (live ? idx : 0);
    const double4 xp = a.sp[m.i_sorted];
    if constexpr (F64) {
        m.hx = live ? xp.x - cx : 1.0e30;
        m.hy = live ? xp.y - cy : 1.0e30;
        m.hz = live ? xp.z - cz : 1.0e30;
        m.mu = xp.w;
        // separations below a tenth of the receiver's offset take the plain
        // form (and r^2 == 0, since ki is at least the smallest normal)
        m.ki = live ? fmax(0.01 * fma(m.hz, m.hz, fma(m.hy, m.hy, m.hx * m.hx)),
                           2.2250738585072014e-308)
                    : 0.0;
        m.rlo = a.g.rc2 * (1.0 - 0x1p-40);
        m.rhi = a.g.rc2 * (1.0 + 0x1p-40);
    } else {
        m.hx = live ? (float)(xp.x - cx) : 1.0e30f;
        m.hy = live ? (float)(xp.y - cy) : 1.0e30f;
        m.hz = live ? (float)(xp.z - cz) : 1.0e30f;
        m.mu = mu_f32(xp.w);
        // separations below a tenth of the receiver's offset are recomputed
        // in FP64 (and r^2 == 0, since ki is at least the smallest normal)
        m.ki = fmaxf(0.01f * fmaf(m.hz, m.hz, fmaf(m.hy, m.hy, m.hx * m.hx)), 1.1754944e-38f);
        if (!live) m.ki = 0.f;
        if constexpr (KIND == kMutSoft) m.eb2 = (float)a.g.eps_b2;
    }
    if constexpr (BWD) {
        if (live) {
            const MutEntry<KIND> wk = MutualVisit<R, UNIT, KIND>::wa_entry_of(a, m.i_sorted);
            m.wkx = wk.x;
            m.wky = wk.y;
            m.wkz = wk.z;
        }
    }
    MutualVisit<R, UNIT, KIND> v{a, m, ring_pos, ring_idx, ring_w, cl.lo, cl.hi, cx, cy, cz,
                                lane, begin + cnt};
    if (item.sole & kItemFirst) v.self_pass(cnt, begin);
    walk_item(v, item, cl, a, lane);
    // the copies of a receiver in the rows r, r + R, ...
    double ax = v.ax, ay = v.ay, az = v.az;
    if constexpr (F64) {
        ax = m.ax;
        ay = m.ay;
        az = m.az;
    }
    if constexpr (R <= 2) {
        ax += __shfl_xor(ax, 32, kWave);
        ay += __shfl_xor(ay, 32, kWave);
        az += __shfl_xor(az, 32, kWave);
    }
    if constexpr (R == 1) {
        ax += __shfl_xor(ax, 16, kWave);
        ay += __shfl_xor(ay, 16, kWave);
        az += __shfl_xor(az, 16, kWave);
    }
    if (row < R && live) {
        atomicAdd(a.out + m.i_sorted, ax);
        atomicAdd(a.out + a.out_stride + m.i_sorted, ay);
        atomicAdd(a.out + 2 * a.out_stride + m.i_sorted, az);
    }
    tally.pairs += v.pairs;
    tally.steps += v.steps;
    tally.screened += v.screened;
    tally.rare += v.rare;
}

// The persistent kernel of the mutual evaluation: clusters of up to 16 RMAX
// receivers, one work item per wave, every particle a receiver.  A cluster
// that fills fewer rows (the last one of a tile is often short) runs in the
// narrower layout, so its receivers meet 16 (4 / R) entries per block with
// fewer idle lanes: 16 receivers or fewer in R = 1, 32 or fewer in R = 2.
// a.out: three FP64 arrays of a.out_stride (= n) values in sorted order,
// zeroed before the launch.
template <int RMAX, bool UNIT, int KIND>
__global__ __launch_bounds__(kForceBlock)
__attribute__((amdgpu_waves_per_eu(kMutIsF64<KIND> ? 4 : 5)))
void k_pairs_mutual(PairArgs a) {
    constexpr bool BWD = kMutIsBwd<KIND>;
    constexpr int NW = kForceBlock / kWave;
    __shared__ MutEntry<KIND> ring_pos[NW][kRing];
    __shared__ int ring_idx[NW][kRing];
    __shared__ MutEntry<KIND> ring_wt[BWD ? NW : 1][BWD ? kRing : 1];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    ItemCursor cursor;
    MutualTally tally;
    const ItemQueue iq = item_queue(a);
    for (int it = next_item(a, iq, lane, cursor); it >= 0; it = next_item(a, iq, lane, cursor)) {
        const Item item = a.items[it];
        const Cluster cl = a.clusters[item.cluster];
        const int cnt = __builtin_amdgcn_readfirstlane(cl.count);
        const int begin = __builtin_amdgcn_readfirstlane(cl.begin);
        if constexpr (RMAX >= 2) {
            if (cnt <= 16) {
                mutual_item<1, UNIT, KIND>(a, item, cl, cnt, begin, lane, ring_pos[w],
                                          ring_idx[w], ring_wt[BWD ? w : 0], tally);
                continue;
            }
        }
        if constexpr (RMAX == 4) {
            if (cnt <= 32) {
                mutual_item<2, UNIT, KIND>(a, item, cl, cnt, begin, lane, ring_pos[w],
                                          ring_idx[w], ring_wt[BWD ? w : 0], tally);
                continue;
            }
        }
        mutual_item<RMAX, UNIT, KIND>(a, item, cl, cnt, begin, lane, ring_pos[w], ring_idx[w],
                                     ring_wt[BWD ? w : 0], tally);
    }
    if (lane == 0 && a.counters && tally.pairs + tally.steps + tally.screened + tally.rare > 0) {
        Counters *k = a.counters + (blockIdx.x % kCounterCopies) * kCounterStride;
        atomicAdd(&k->interactions, tally.pairs);
        atomicAdd(&k->steps, tally.steps);
        atomicAdd(&k->screened, tally.screened);
        atomicAdd(&k->rare, tally.rare);
    }
}

// acc_out[3 perm[p] + c] = sums[c n + p]
__global__ void k_mutual_out(const double *__restrict__ sums, const int *__restrict__ perm, int n,
                             double *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const size_t o = 3 * (size_t)perm[p];
    out[o] = sums[p];
    out[o + 1] = sums[(size_t)n + p];
    out[o + 2] = sums[2 * (size_t)n + p];
}

using MutualFn = void (*)(PairArgs);

template <int KIND>
MutualFn mutual_kernel_mode(int csize, bool unit) {
    switch (csize) {
    case 16: return unit ? k_pairs_mutual<1, true, KIND> : k_pairs_mutual<1, false, KIND>;
    case 32: return unit ? k_pairs_mutual<2, true, KIND> : k_pairs_mutual<2, false, KIND>;
    case 64: return unit ? k_pairs_mutual<4, true, KIND> : k_pairs_mutual<4, false, KIND>;
    default: return nullptr;
    }
}

// soft: the forward with B-spline softening (the adjoint has no softened
// mutual kernel); f64: the FP64 kinds (likewise)
MutualFn mutual_kernel(int csize, bool unit, bool bwd, bool soft, bool f64) {
    if (f64) {
        if (bwd) return soft ? nullptr : mutual_kernel_mode<kMutF64Bwd>(csize, unit);
        return soft ? mutual_kernel_mode<kMutF64Soft>(csize, unit) : mutual_kernel_mode<kMutF64>(csize, unit);
    }
    if (bwd) return soft ? nullptr : mutual_kernel_mode<kMutBwd>(csize, unit);
    return soft ? mutual_kernel_mode<kMutSoft>(csize, unit) : mutual_kernel_mode<kMutFwd>(csize, unit);
}

// The pair-kernel variant for a layout: all share the signature void(PairArgs).
using PairsFn = void (*)(PairArgs);

template <int MODE, bool UNIT, bool SOFT, int TAB = SHAPE_POLY>
PairsFn pairs_fn_sg(int sg) {
    switch (sg) {
    case 1: return k_pairs<MODE, UNIT, 1, SOFT, TAB>;
    case 2: return k_pairs<MODE, UNIT, 2, SOFT, TAB>;
    case 4: return k_pairs<MODE, UNIT, 4, SOFT, TAB>;
    case 8: return k_pairs<MODE, UNIT, 8, SOFT, TAB>;
    default: return k_pairs<MODE, UNIT, 0, SOFT, TAB>;
    }
}

template <int MODE, bool UNIT>
PairsFn pairs_fn_soft(int sg, bool soft) {
    return soft ? pairs_fn_sg<MODE, UNIT, true>(sg) : pairs_fn_sg<MODE, UNIT, false>(sg);
}

// screen groups: 64 / csize when screening (csize in {8, 16, 32, 64}), else 0
inline int screen_groups(int screen, int csize) { return screen ? kWave / csize : 0; }

// H at t = u^2 in FP64 from the degree-17 interpolant (error 1.5e-15 in g).
__global__ void k_build_htab(int kind, int n, Geom g, float *tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (kind == SHAPE_TAB_NGP) {
        const double r2 = ((double)k + 0.5) * g.rc2 / (double)n;
        tab[k] = (float)h64(r2 * g.c2 - P3M_H64_T0, g.h64);
    } else {
        const double h0 = h64((double)k * g.rc2 / (double)n * g.c2 - P3M_H64_T0, g.h64);
        const double h1 = h64((double)(k + 1) * g.rc2 / (double)n * g.c2 - P3M_H64_T0, g.h64);
        tab[2 * k] = (float)h0;
        tab[2 * k + 1] = (float)(h1 - h0);
    }
}

}  // namespace

hipError_t launch_build_htab(int kind, int n, const Geom &g, float *tab, hipStream_t s) {
    k_build_htab<<<(n + 255) / 256, 256, 0, s>>>(kind, n, g, tab);
    return hipGetLastError();
}

// The kernel that launch_pairs runs for this call (nullptr: invalid layout).
// The FP32 forward with the tabulated shape exists without softening only.
static PairsFn pairs_kernel(int mode, int screen, int tab, int csize, bool unit, bool soft) {
    if (csize != 8 && csize != 16 && csize != 32 && csize != 64) return nullptr;
    const int sg = screen_groups(screen, csize);
    switch (mode) {
    case FWD_F32:
        if (tab != SHAPE_POLY && !soft) {
            if (tab == SHAPE_TAB_NGP)
                return unit ? pairs_fn_sg<FWD_F32, true, false, SHAPE_TAB_NGP>(sg)
                            : pairs_fn_sg<FWD_F32, false, false, SHAPE_TAB_NGP>(sg);
            return unit ? pairs_fn_sg<FWD_F32, true, false, SHAPE_TAB_LINEAR>(sg)
                        : pairs_fn_sg<FWD_F32, false, false, SHAPE_TAB_LINEAR>(sg);
        }
        return unit ? pairs_fn_soft<FWD_F32, true>(sg, soft) : pairs_fn_soft<FWD_F32, false>(sg, soft);
    case FWD_F64:
        return unit ? pairs_fn_soft<FWD_F64, true>(sg, soft) : pairs_fn_soft<FWD_F64, false>(sg, soft);
    case BWD_F32: return pairs_fn_soft<BWD_F32, false>(sg, soft);
    default: return pairs_fn_soft<BWD_F64, false>(sg, soft);
    }
}

hipError_t launch_pairs(int mode, int screen, int tab, const PairArgs &a, int grid,
                        hipStream_t s) {
    const bool soft = a.g.eps_b > 0.0;
    if (mode == FWD_F32 && tab != SHAPE_POLY && !soft) {
        const int nf = tab == SHAPE_TAB_LINEAR ? 2 * a.tab_n : a.tab_n;
        if (!a.htab || a.tab_n < 1 || nf > kTabFloats) return hipErrorInvalidValue;
    }
    const bool unit = a.unit_mass && (mode == FWD_F32 || mode == FWD_F64);
    const PairsFn fn = pairs_kernel(mode, screen, tab, a.csize, unit, soft);
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kForceBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pairs_mutual(const PairArgs &a, bool bwd, bool f64, int grid, hipStream_t s) {
    const MutualFn fn = mutual_kernel(a.csize, a.unit_mass != 0, bwd, a.g.eps_b > 0.0, f64);
    if (!fn) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kForceBlock), 0, s, a);
    return hipGetLastError();
}

int mutual_blocks_per_cu(int csize, int unit_mass, bool bwd, bool soft, bool f64) {
    const MutualFn fn = mutual_kernel(csize, unit_mass != 0, bwd, soft, f64);
    int nb = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kForceBlock, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_mutual_out(const double *sums, const int *perm, int n, double *out,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mutual_out, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sums,
                       perm, n, out);
    return hipGetLastError();
}

// Blocks of the persistent grid per CU.  The six-wave FP32 variant is sized
// by its own limit (6).  Every other variant is sized by what the largest
// screened variant of its mode and softening (per-particle masses, 8-receiver
// clusters: the most registers) leaves room for, as if it were launched: for
// FP64 that is 4 blocks, against the 5 the unit-mass variant would fit, and 4
// measured 2 % faster.
int pairs_blocks_per_cu(int mode, int screen, int tab, int csize, int unit_mass, int soft) {
    bool unit = unit_mass && (mode == FWD_F32 || mode == FWD_F64);
    const bool six = mode == FWD_F32 && unit && tab == SHAPE_POLY && !soft;
    if (!six) {
        unit = false;
        screen = screen ? 1 : 0;
        if (screen) csize = 8;
    }
    const PairsFn fn = pairs_kernel(mode, screen, tab, csize, unit, soft != 0);
    int nb = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kForceBlock, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

}  // namespace p3m
