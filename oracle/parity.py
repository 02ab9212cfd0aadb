"""Parity of GPU supersegment lists with the oracle's outcomes (shared by the
GPU tests and the benchmark's CPU-baseline comparison).  Test
infrastructure, like the rest of this package.

The oracle decides every Eq. 1 branch in fp64.  Where a decision's distance
lies within the near-tie band of gamma (oracle.TIE, widened for long
supersegments), an fp32 implementation may take the other branch, so the
oracle enumerates every outcome its near ties admit: the fp64 one in the
regular outputs and the others in "alts" ("nout" per list: the number of
outcomes, negative when the enumeration was cut short).  A GPU list passes
when it equals one of them: the same count and threshold, and every stored
value within ATOL.  Every list, whatever its outcome count, must also satisfy
the invariants of a VDI list (count within N, f < b, fronts non-decreasing,
colours and opacities in [0, 1]).
"""
from __future__ import annotations

import numpy as np

ATOL = 1e-5


def _match(gc, gd, gn, gg, oc, od, on, og, N):
    """Per list: equal (clamped) count and threshold, stored slots within ATOL.
    gc [N, M, 4], gd [N, M, 2], gn [M], gg [M] or None; oc, od, on, og alike."""
    on = np.minimum(on, N)
    ok = gn == on
    if gg is not None and og is not None:
        ok &= gg == og
    used = np.arange(N)[:, None] < on[None, :]
    dc = np.where(used[..., None], np.abs(gc - oc), 0.0).max(axis=(0, 2), initial=0.0)
    dd = np.where(used[..., None], np.abs(gd - od), 0.0).max(axis=(0, 2), initial=0.0)
    return ok & (dc <= ATOL) & (dd <= ATOL), np.maximum(dc, dd)


def invariants(gc, gd, gn, N, label):
    """Checks every list: 0 <= count <= N, zeros beyond the count, f < b and
    finite, fronts non-decreasing, colours and opacities in [0, 1]."""
    assert gn.min(initial=0) >= 0 and gn.max(initial=0) <= N, f"{label}: count outside [0, {N}]"
    used = np.arange(N)[:, None] < gn[None, :]
    assert np.all(gc[~used] == 0) and np.all(gd[~used] == 0), f"{label}: slots beyond the count not zero-filled"
    f, b = gd[..., 0], gd[..., 1]
    assert np.all(np.isfinite(gd[used])) and np.all(f[used] < b[used]), f"{label}: f < b violated"
    if N > 1:
        step = used[1:] & (f[1:] < f[:-1])
        assert not step.any(), f"{label}: fronts decrease"
    c = gc[used]
    assert np.all((c >= 0.0) & (c <= 1.0 + 1e-6)), f"{label}: colour or opacity outside [0, 1]"


def check_lists(gpu, ref, label, brick=None, use_gamma=True, max_incomplete=1e-3, invariant=True, strict=True,
                masks=False):
    """GPU lists (color [N, P, 4], depth [N, P, 2], count [P], gamma [P] or
    None) against the oracle's outcomes `ref` (generation: brick `brick` of
    it; composite: brick None).  Returns counts of lists matched by the fp64
    outcome, by another near-tie outcome, and left unresolved because their
    enumeration was cut short (allowed up to max_incomplete of the non-empty
    lists; they are checked by the invariants).  strict=False reports lists
    matching no outcome as "mismatch" instead of raising; masks=True adds the
    per-list "fp64_mask" (matched the fp64 outcome)."""
    gc, gd, gn, gg = gpu
    N, P = gc.shape[0], gc.shape[1]
    if brick is None:
        oc, od, on, og, no, base = ref["color"], ref["depth"], ref["count"], ref["gamma"], ref["nout"], 0
    else:
        oc, od, on = ref["color"][brick], ref["depth"][brick], ref["count"][brick]
        og, no, base = ref["gamma"][brick], ref["nout"][brick], brick * P
    if not use_gamma:
        gg = og = None
    if invariant:
        invariants(gc, gd, gn, N, label)
    ok, err = _match(gc, gd, gn, gg, oc, od, on, og, N)
    by_alt = np.zeros(P, bool)
    alts = ref["alts"]
    miss = np.nonzero(~ok)[0]
    if len(miss):
        rays = alts["ray"] - base
        for q in miss:
            rows = np.nonzero(rays == q)[0]
            if not len(rows):
                continue
            ac = alts["color"][rows].transpose(1, 0, 2)
            ad = alts["depth"][rows].transpose(1, 0, 2)
            m, _ = _match(np.repeat(gc[:, q:q + 1], len(rows), 1), np.repeat(gd[:, q:q + 1], len(rows), 1),
                          np.repeat(gn[q:q + 1], len(rows)), None if gg is None else np.repeat(gg[q:q + 1], len(rows)),
                          ac, ad, alts["count"][rows], None if og is None else alts["gamma"][rows], N)
            by_alt[q] = m.any()
    unresolved = ~ok & ~by_alt
    incomplete = no < 0
    bad = unresolved & ~incomplete
    if bad.any() and strict:
        q = int(np.nonzero(bad)[0][0])
        raise AssertionError(
            f"{label}: {int(bad.sum())} lists match no oracle outcome (e.g. list {q}: gpu count {gn[q]} "
            f"gamma {None if gg is None else gg[q]}, oracle count {on[q]} gamma {og[q] if og is not None else None}, "
            f"outcomes {no[q]}, max value error {err[q]:.3g})")
    nonempty = max(int(((on > 0) | (gn > 0)).sum()), 1)
    unres = int((unresolved & incomplete).sum())
    if strict:
        assert unres <= max_incomplete * nonempty, f"{label}: {unres} lists with an incomplete outcome enumeration"
    out = {"lists": P, "nonempty": nonempty, "fp64_outcome": int(ok.sum()), "near_tie_outcome": int(by_alt.sum()),
           "several_outcomes": int((no >= 2).sum()), "unresolved_incomplete": unres, "mismatch": int(bad.sum())}
    if masks:
        out["fp64_mask"] = ok
    return out
