// Rung-hierarchical kick-drift-kick step (CONCEPT 1.0, section 2.2.2,
// "Individual time steps", the time-stepping figure and eq. rung) in a
// static box: drift x += v tau, kick v += a dt_kick.
//
// Time is counted in integer units of tau / 2, tau = dt / 2^L the drift
// sub-step (L the highest rung of the period).  Rung l kicks every
// span(l) = 2^(L+1-l) units.  Each particle carries the time of its
// momentum (t_q) and of its next kick (t_next); a kick at time t brings the
// momentum to t + span(rung) / 2, or to the period's end at the last kick.
// The host loop (api.hip) drifts, marks the particles due at t, evaluates the
// short-range force with them as receivers and calls k_kdk_kick; the
// long-range force is added to everyone whenever rung 0 kicks.
#include <hip/hip_runtime.h>

#include "p3msr_internal.hpp"

namespace p3m {
namespace {

// eq. rung: max(0, ceil(log2(dt sqrt(|a| / (2 eta eps))))), capped.  The
// ceiling of log2 is read off the binary exponent, exactly.
__device__ __forceinline__ int rung_of(double ax, double ay, double az, const KdkArgs &k) {
    const double mag = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(ax, ax), __dmul_rn(ay, ay)),
                                      __dmul_rn(az, az)));
    if (!(mag > 0.0)) return 0;
    const double z = k.dt * sqrt(mag / k.two_eta_eps);
    int e;
    const double m = frexp(z, &e);   // z = m 2^e, m in [0.5, 1)
    int l = m == 0.5 ? e - 1 : e;
    l = l < 0 ? 0 : l;
    return l > k.max_rung ? k.max_rung : l;
}

__device__ __forceinline__ int span_of(int l, int L) { return 1 << (L + 1 - l); }

__global__ void k_kdk_assign(const double *__restrict__ acc, int n, KdkArgs k,
                             uint8_t *__restrict__ rung, int *__restrict__ max_rung) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int l;
    if (k.fixed) {
        l = rung[i];
    } else {
        l = rung_of(acc[3 * (size_t)i], acc[3 * (size_t)i + 1], acc[3 * (size_t)i + 2], k);
        rung[i] = (uint8_t)l;
    }
    atomicMax(max_rung, l);
}

// The half kicks from the synchronised start.
__global__ void k_kdk_first(double *__restrict__ vel, const double *__restrict__ acc, int n,
                            KdkArgs k, const uint8_t *__restrict__ rung, int *__restrict__ t_q,
                            int *__restrict__ t_next) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sp = span_of(rung[i], k.L);
    const int target = sp / 2;
    const double dk = (double)target * k.half_tau;
    for (int d = 0; d < 3; ++d) vel[3 * (size_t)i + d] = vel[3 * (size_t)i + d] + acc[3 * (size_t)i + d] * dk;
    t_q[i] = target;
    t_next[i] = sp;
}

__global__ void k_kdk_drift(double *__restrict__ pos, const double *__restrict__ vel, size_t n3,
                            double tau, double box) {
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n3) return;
    double x = pos[j] + vel[j] * tau;
    double r = fmod(x, box);
    if (r < 0.0) r += box;
    if (r >= box) r -= box;
    pos[j] = r;
}

__global__ void k_kdk_due(const int *__restrict__ t_next, int n, int t, uint8_t *__restrict__ due,
                          int *__restrict__ n_due) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool d = t_next[i] == t;
    due[i] = (uint8_t)d;
    // one atomic per wave
    const unsigned long long b = __ballot(d);
    if (b && (threadIdx.x & (kWave - 1)) == (unsigned)(__ffsll((long long)b) - 1))
        atomicAdd(n_due, __popcll(b));
}

__global__ void k_kdk_kick(double *__restrict__ vel, const double *__restrict__ acc,
                           const uint8_t *__restrict__ due, int n, int t, KdkArgs k,
                           uint8_t *__restrict__ rung, int *__restrict__ t_q,
                           int *__restrict__ t_next) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !due[i]) return;
    const double ax = acc[3 * (size_t)i], ay = acc[3 * (size_t)i + 1], az = acc[3 * (size_t)i + 2];
    int l = rung[i];
    const bool last = t == k.period;
    const int target = last ? k.period : t + span_of(l, k.L) / 2;
    const double dk = (double)(target - t_q[i]) * k.half_tau;
    vel[3 * (size_t)i] = vel[3 * (size_t)i] + ax * dk;
    vel[3 * (size_t)i + 1] = vel[3 * (size_t)i + 1] + ay * dk;
    vel[3 * (size_t)i + 2] = vel[3 * (size_t)i + 2] + az * dk;
    t_q[i] = target;
    if (k.fixed) {
        if (!last) t_next[i] = t + span_of(l, k.L);
        return;
    }
    const int want = rung_of(ax, ay, az, k);
    if (last) {
        rung[i] = (uint8_t)want;   // the next period's rung (uncapped by L)
        return;
    }
    const int w = want < k.L ? want : k.L;
    if (w > l) {
        l = l + 1;
    } else if (w < l && (t + span_of(l, k.L)) % span_of(l - 1, k.L) == 0) {
        l = l - 1;
    }
    rung[i] = (uint8_t)l;
    const int sp = span_of(l, k.L);
    t_next[i] = (t / sp + 1) * sp;
}

// y += a x over n x 3 values (long-range kicks; summing the two force halves)
__global__ void k_axpy3(double *__restrict__ vel, const double *__restrict__ acc, size_t n3,
                        double dk) {
    const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n3) return;
    vel[j] = vel[j] + acc[j] * dk;
}

// Adds one force call's accepted-pair count (the sum of its counter copies)
// to the period's total.
__global__ void k_kdk_accum(const Counters *__restrict__ c, unsigned long long *__restrict__ total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long s = 0;
        for (int k = 0; k < kCounterCopies; ++k) s += c[k * kCounterStride].interactions;
        *total += s;
    }
}

unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_kdk_assign(const double *acc, int n, const KdkArgs &k, uint8_t *rung,
                             int *max_rung, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_kdk_assign<<<blocks(n), 256, 0, s>>>(acc, n, k, rung, max_rung);
    return hipGetLastError();
}

hipError_t launch_kdk_first(double *vel, const double *acc, int n, const KdkArgs &k,
                            const uint8_t *rung, int *t_q, int *t_next, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_kdk_first<<<blocks(n), 256, 0, s>>>(vel, acc, n, k, rung, t_q, t_next);
    return hipGetLastError();
}

hipError_t launch_kdk_drift(double *pos, const double *vel, int n, double tau, double box,
                            hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_kdk_drift<<<blocks(3 * (size_t)n), 256, 0, s>>>(pos, vel, 3 * (size_t)n, tau, box);
    return hipGetLastError();
}

hipError_t launch_kdk_due(const int *t_next, int n, int t, uint8_t *due, int *n_due,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_kdk_due<<<blocks(n), 256, 0, s>>>(t_next, n, t, due, n_due);
    return hipGetLastError();
}

hipError_t launch_kdk_kick(double *vel, const double *acc, const uint8_t *due, int n, int t,
                           const KdkArgs &k, uint8_t *rung, int *t_q, int *t_next,
                           hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_kdk_kick<<<blocks(n), 256, 0, s>>>(vel, acc, due, n, t, k, rung, t_q, t_next);
    return hipGetLastError();
}

hipError_t launch_axpy3(double *vel, const double *acc, int n, double dk, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_axpy3<<<blocks(3 * (size_t)n), 256, 0, s>>>(vel, acc, 3 * (size_t)n, dk);
    return hipGetLastError();
}

hipError_t launch_kdk_accum(const Counters *c, unsigned long long *total, hipStream_t s) {
    k_kdk_accum<<<1, 64, 0, s>>>(c, total);
    return hipGetLastError();
}

}  // namespace p3m
