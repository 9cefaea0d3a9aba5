"""Host model of the near-field kernel's work split (no GPU): a target leaf's
near-list source ranges are concatenated into passes of at most LIST point
indices staged in shared memory; targets run in blocks of up to 64 with
lane = t + nt q for source slice q of S = 64 / nt; slice q takes the pass's
sources q, q + S, .. two per step.  Every (target, source) pair of the leaf
must be evaluated exactly once, by the lane of its target, and each slice
must take its sources in concatenated order, so that the sums are
deterministic."""
import numpy as np
import pytest


def leaf_visits(ranges, n_targets, LIST):
    """(target, source) pairs in the order each lane adds them."""
    tot = sum(e - s for s, e in ranges)
    visits = {}
    for ib in range(0, n_targets, 64):
        nt = min(64, n_targets - ib)
        S = 64 // nt
        for v0 in range(0, tot, LIST):
            nv = min(LIST, tot - v0)
            lst = [None] * nv
            cum = 0
            for a, b in ranges:  # staging, as the kernel's lanes write it
                if cum >= v0 + nv:
                    break
                ln = b - a
                lo, hi = max(v0 - cum, 0), min(v0 + nv - cum, ln)
                for lane in range(64):
                    for l in range(lo + lane, hi, 64):
                        lst[cum + l - v0] = a + l
                cum += ln
            assert all(x is not None for x in lst)
            for lane in range(64):
                q, t = lane // nt, lane - (lane // nt) * nt
                if q >= S:
                    continue
                v = q
                while v + S < nv:
                    visits.setdefault((ib + t, q), []).extend([lst[v], lst[v + S]])
                    v += 2 * S
                if v < nv:
                    visits.setdefault((ib + t, q), []).append(lst[v])
    return visits


@pytest.mark.parametrize("n_targets,LIST", [(1, 2048), (7, 2048), (22, 16), (33, 2048), (64, 40), (100, 13)])
def test_every_pair_once_in_slice_order(n_targets, LIST):
    rng = np.random.default_rng(n_targets + LIST)
    ranges, start = [], 0
    for _ in range(int(rng.integers(1, 12))):
        start += int(rng.integers(0, 50))
        ln = int(rng.integers(1, 30))
        ranges.append((start, start + ln))
        start += ln
    flat = [j for a, b in ranges for j in range(a, b)]
    visits = leaf_visits(ranges, n_targets, LIST)
    for t in range(n_targets):
        S = 64 // min(64, n_targets - (t // 64) * 64)
        got = []
        for q in range(S):
            seq = visits.get((t, q), [])
            # slice q: concatenated sources q, q + S, .. within every pass, in order
            expect = [flat[v0 + v] for v0 in range(0, len(flat), LIST)
                      for v in range(q, min(LIST, len(flat) - v0), S)]
            assert seq == expect, (t, q)
            got.extend(seq)
        assert sorted(got) == sorted(flat), t
