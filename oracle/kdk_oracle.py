"""Plain FP64 oracle of the rung-hierarchical kick-drift-kick step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU legs are the only callers.  The GPU library never imports
this module and this module never imports the GPU library.

What is computed (CONCEPT 1.0, section 2.2.2, "Individual time steps", the
time-stepping figure and eq. rung), in a static box (scale factor 1, so the
drift and kick integrals of the D and K operators are plain durations and
q / m is the velocity v):

  * One call advances a synchronised state (x, v at the same time) by
    n_steps global steps dt and synchronises it again at the end (the
    paper's period of steps between synchronisations).
  * At the start every particle gets a rung from eq. rung,
        rung = max(0, ceil(log2(dt sqrt(|a| / (2 eta eps))))),
    capped at max_rung, where |a| is its short-range acceleration at the
    start (a force evaluation whose momentum update is not applied).  L is the
    highest rung; positions drift in sub-steps tau = dt / 2^L.
  * Rung l kicks every dt / 2^l.  A kick at time t with the particle on
    rung l brings its momentum from wherever it is to t + dt / 2^(l+1)
    (half a step of its rung ahead); the very first kick is the half kick
    from the synchronised start, and the kick at the period's end brings
    every momentum back to the end time.  Kicks use the short-range force
    only, with the kicked particles as receivers and all particles as
    suppliers.
  * After each kick inside the period the particle's rung is re-evaluated
    from the short-range acceleration of that kick: it moves at most one
    rung up, or one rung down only when its next kick time is also a kick
    time of the lower rung; its next kick is at the next kick time of its
    new rung.  Measuring momentum time per particle makes the next kick
    after a jump half (up) or three quarters (down) of the new rung's usual
    kick, as the paper describes.
  * The long-range force is applied to all particles whenever rung 0 is
    kicked: half kicks at the two ends of the period, full ones between.
  * At the end the rungs are re-assigned from the final short-range
    accelerations (the next period's start).

Time is counted in integer units of tau / 2, so every kick target is exact.
"""
from __future__ import annotations

import math

import numpy as np


def rung_of(acc, dt, eta, eps, max_rung):
    """eq. rung for each row of acc (n x 3), capped at max_rung."""
    out = np.zeros(acc.shape[0], dtype=np.int64)
    for i, a in enumerate(acc):
        mag = math.sqrt(float(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]))
        if mag == 0.0:
            continue
        z = dt * math.sqrt(mag / (2.0 * eta * eps))
        out[i] = min(max(0, math.ceil(math.log2(z))), max_rung)
    return out


def kdk(pos, vel, box, dt, n_steps, force_sr, force_lr=None, *, eta=0.025, eps=None,
        rung=None, fixed_rungs=False, max_rung=7, log=None):
    """Advance (pos, vel) by n_steps steps of dt; returns (pos, vel, rung_out).

    force_sr(pos, receivers) -> (n, 3) short-range accelerations of the
    particles flagged in the uint8 mask `receivers` (other rows unused);
    force_lr(pos) -> (n, 3) long-range accelerations, or None.
    With fixed_rungs the input `rung` is used throughout and returned
    unchanged; otherwise rungs follow eq. rung (eps > 0 needed).
    log, if a list, receives (particle, time, kick duration) for every
    short-range kick."""
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    n = x.shape[0]
    everyone = np.ones(n, dtype=np.uint8)
    a_sr = force_sr(x, everyone)
    if fixed_rungs:
        r = np.asarray(rung, dtype=np.int64).copy()
    else:
        r = rung_of(a_sr, dt, eta, eps, max_rung)
    L = int(r.max()) if n else 0
    tau = dt / 2 ** L
    half_tau = 0.5 * tau
    period = n_steps * 2 ** (L + 1)                 # in units of tau / 2

    def span(l):                                    # kick interval of rung l, in tau / 2
        return 2 ** (L + 1 - l)

    # the half kicks from the synchronised start
    t_q = np.zeros(n, dtype=np.int64)               # time of each momentum
    t_next = np.zeros(n, dtype=np.int64)
    for i in range(n):
        target = span(r[i]) // 2
        dk = (target - t_q[i]) * half_tau
        v[i] = v[i] + a_sr[i] * dk
        if log is not None:
            log.append((i, 0, dk))
        t_q[i] = target
        t_next[i] = span(r[i])
    t_lr = 0
    if force_lr is not None:
        target = span(0) // 2
        v = v + force_lr(x) * ((target - t_lr) * half_tau)
        t_lr = target

    for t in range(2, period + 1, 2):
        x = x + v * tau                              # drift all by tau
        x = x % box
        x[x >= box] -= box
        due = (t_next == t).astype(np.uint8)
        if due.any():
            a_sr = force_sr(x, due)         # at t == period every particle is due
            if not fixed_rungs and t < period:
                r_new = rung_of(a_sr, dt, eta, eps, max_rung)
            for i in np.nonzero(due)[0]:
                target = period if t == period else t + span(r[i]) // 2
                dk = (target - t_q[i]) * half_tau
                v[i] = v[i] + a_sr[i] * dk
                if log is not None:
                    log.append((i, t, dk))
                t_q[i] = target
                if t == period:
                    continue
                l = r[i]
                if not fixed_rungs:
                    want = min(int(r_new[i]), L)
                    if want > l:
                        l = l + 1
                    elif want < l and (t + span(l)) % span(l - 1) == 0:
                        l = l - 1
                r[i] = l
                t_next[i] = (t // span(l) + 1) * span(l)
        if force_lr is not None and t % span(0) == 0:
            target = period if t == period else t + span(0) // 2
            v = v + force_lr(x) * ((target - t_lr) * half_tau)
            t_lr = target
    if not fixed_rungs:
        r = rung_of(a_sr, dt, eta, eps, max_rung)
    return x, v, r
