"""Brute-force lineage simulation of a cascade in a frozen field (test helper).

With zero macro-particle weight the current vanishes and E stays at its
uniform initial value, so every lepton evolves on its own.  This helper
follows each lepton from its birth to the end of the run, one lineage at a
time (depth first), and draws its photons with its own Philox4x32-10 (written
here from the published definition and pinned to the generator's published
known-answer vectors) rather than the oracle's generator.  Counting births, deaths and conversions per
step then gives the per-step totals the oracle must reproduce exactly.

The emission model is that of section 2 of arXiv:2012.05587 (threshold
gamma_thr, pair energy f*gamma_thr split equally, emitter direction kept),
optionally with a per-lepton spread of the threshold;
the photon path and the fixed-point move are the readings documented in the
oracle.
"""
import math

import numpy as np

TAG_PHOTON = 2
TAG_THRESHOLD = 3


def philox(ctr, key):
    """Philox4x64-10 block for counter ``ctr`` (numpy bumps the counter first)."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    v = (v - 1) % (1 << 256)
    cc = np.array([(v >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=cc)
    return [int(x) for x in bg.random_raw(4)]


_M32 = 0xFFFFFFFF


def philox4x32(ctr, key):
    """Philox4x32-10 block: ten rounds of two 32 x 32 -> 64-bit products by
    0xD2511F53 (word 0) and 0xCD9E8D57 (word 2), the new words being
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by 0x9E3779B9
    and 0xBB67AE85 before every round after the first."""
    c0, c1, c2, c3 = (int(x) & _M32 for x in ctr)
    k0, k1 = (int(x) & _M32 for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & _M32
            k1 = (k1 + 0xBB67AE85) & _M32
        a = 0xD2511F53 * c0
        b = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = (b >> 32) ^ c1 ^ k0, b & _M32, (a >> 32) ^ c3 ^ k1, a & _M32
    return [c0, c1, c2, c3]


def draw_run(pid, seed, step, j, tag):
    """A lepton's draw during the run: counter (step, j | tag << 8, id low, id
    high), key (seed low, seed high); returns (words 1:0 as 64 bits, word 2)."""
    w = philox4x32((step, j | (tag << 8), pid & _M32, pid >> 32), (seed & _M32, seed >> 32))
    return (w[1] << 32) | w[0], w[2]


def conv_table(dt, dx, l_gamma):
    r = dt / (l_gamma * dx)
    t = []
    k = 0
    while True:
        v = math.floor(math.ldexp(math.exp(-(k * r)), 32))
        t.append(v)
        k += 1
        if v == 0:
            return t


def threshold(pid, seed, gamma_thr, spread):
    """A lepton's own threshold under a spread of gamma_thr: uniform in
    gamma_thr (1 - spread, 1 + spread) from the top 53 bits of the 64-bit value
    of its tag-3 draw, in binary64."""
    bits, _ = draw_run(pid, seed, 0, 0, TAG_THRESHOLD)
    x = (bits >> 11) * 2.0 ** -53
    return gamma_thr * (1.0 + spread * (2.0 * x - 1.0))


def run(n_cells, dx, dt, absorbing, e0, gamma_thr, f, l_gamma, seeds, n_steps, seed,
        gamma_thr_spread=0.0):
    """seeds: list of (species, cell, offq, p, id) with offq in units of 2^-40.

    Returns per-step totals and the final leptons {id: (species, cell, offq, p)}.
    """
    K = 40
    ONE = 1 << K
    dtdx = dt / dx
    gpair = f * gamma_thr
    ghalf = gpair * 0.5
    pchild = math.sqrt(ghalf * ghalf - 1.0)
    photon_step = round(math.ldexp(dt / dx, K))
    domain = n_cells * ONE
    table = conv_table(dt, dx, l_gamma) if l_gamma > 0 else None

    alive = np.zeros((2, n_steps), dtype=np.int64)   # leptons alive after step n
    inflight = np.zeros(n_steps, dtype=np.int64)
    emitted = np.zeros(n_steps, dtype=np.int64)
    escaped = np.zeros(n_steps, dtype=np.int64)
    created = np.zeros(n_steps, dtype=np.int64)
    absorbed = np.zeros((2, n_steps), dtype=np.int64)
    final = {}

    # stack of leptons to follow: (species, cell, offq, p, id, first step pushed)
    stack = [(s, c, o, p, i, 0) for (s, c, o, p, i) in seeds]
    # leptons present before step 0 count as alive from step 0 until they die
    while stack:
        s, c, oq, p, pid, first = stack.pop()
        q = -1 if s == 0 else 1
        qdt = q * dt
        died_at = None
        thr = (threshold(pid, seed, gamma_thr, gamma_thr_spread) if gamma_thr_spread > 0.0
               else gamma_thr)
        for n in range(first, n_steps):
            # uniform field: the node average and the interpolation give E0
            p = p + qdt * e0
            gam = math.sqrt(1.0 + p * p)
            v = p / gam
            d = v * dtdx
            nq = oq + round(d * ONE)
            if nq >= ONE:
                nq -= ONE
                c += 1
            elif nq < 0:
                nq += ONE
                c -= 1
            if c < 0 or c >= n_cells:
                if absorbing:
                    absorbed[s, n:] += 1
                    died_at = n
                    break
                c %= n_cells
            oq = nq
            gm = gam
            k = 0
            while gm >= thr:
                gm = gm - gpair
                k += 1
            if k:
                mag = math.sqrt(gm * gm - 1.0)
                direction = 1 if p > 0 else -1
                p = mag if direction > 0 else -mag
                for j in range(k):
                    bits, u32 = draw_run(pid, seed, n, j, TAG_PHOTON)
                    child = bits & ~1
                    emitted[n:] += 1
                    if table is None:
                        created[n:] += 1
                        if n + 1 < n_steps:
                            stack.append((0, c, oq, direction * pchild, child, n + 1))
                            stack.append((1, c, oq, direction * pchild, child | 1, n + 1))
                        else:
                            final[child] = (0, c, oq, direction * pchild)
                            final[child | 1] = (1, c, oq, direction * pchild)
                            alive[0, n] += 1
                            alive[1, n] += 1
                        continue
                    nconv = next(kk for kk in range(1, len(table)) if u32 >= table[kk])
                    X = c * ONE + oq + direction * nconv * photon_step
                    if absorbing and (X < 0 or X >= domain):
                        escaped[n:] += 1
                        continue
                    X %= domain
                    conv = n + nconv
                    inflight[n:min(conv, n_steps)] += 1
                    if conv < n_steps:
                        created[conv:] += 1
                        cc, co = X // ONE, X % ONE
                        if conv + 1 < n_steps:
                            stack.append((0, cc, co, direction * pchild, child, conv + 1))
                            stack.append((1, cc, co, direction * pchild, child | 1, conv + 1))
                        else:
                            final[child] = (0, cc, co, direction * pchild)
                            final[child | 1] = (1, cc, co, direction * pchild)
                            alive[0, conv] += 1
                            alive[1, conv] += 1
            alive[s, n] += 1
        if died_at is None and first < n_steps:
            final[pid] = (s, c, oq, p)
        # a lepton born at the end of step first-1 is alive after that step too
        if first > 0:
            alive[s, first - 1] += 1
    return {"n_minus": alive[0], "n_plus": alive[1], "n_photons": inflight,
            "photons_emitted": emitted, "photons_escaped": escaped,
            "pairs_created": created, "absorbed_minus": absorbed[0],
            "absorbed_plus": absorbed[1], "final": final}
