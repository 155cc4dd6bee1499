"""Radiance bars of the generation parity tests (GPU light field against the
FP64 oracle on the same random stream).

  - aggregate relative L1, sum |gpu - ref| / sum |ref| over the compared
    texels and channels: <= 1e-3 (the bar set for this path);
  - flips: a value whose relative error exceeds 1e-2 (with |ref| floored at
    1e-3 of the mean radiance) comes from a sample in which an FP32 decision
    (a delta-tracking accept, a slab exit, a cell crossing) went the other
    way than the FP64 one, which replaces that whole sample.  Their share of
    the compared values is bounded per workload at a few times the measured
    rate, so that a tenfold rise fails;
  - the 99th percentile of the per-value relative error (same floor) stays
    below 1e-3: outside the flips the two sides agree to FP32 rounding of
    the sample sums.
"""
import numpy as np

RAD_TOL = 1e-3
FLIP_REL = 1e-2
P99_TOL = 1e-3


def report(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    floor = 1e-3 * np.abs(ref).mean()
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
    return {"rel_l1": float(np.abs(got - ref).sum() / np.abs(ref).sum()),
            "flip_frac": float((rel > FLIP_REL).mean()),
            "p99_rel": float(np.quantile(rel, 0.99)),
            "mean_rel": float(rel.mean()),
            "max_rel": float(rel.max()),
            "values": int(rel.size)}


def check(got, ref, flip_max, label="", rel_l1_max=RAD_TOL):
    r = report(got, ref)
    print(f"{label}: rel L1 {r['rel_l1']:.3e}, flips {r['flip_frac']:.2e} of {r['values']} values "
          f"(bound {flip_max:.1e}), p99 {r['p99_rel']:.2e}, mean {r['mean_rel']:.2e}, max {r['max_rel']:.2e}")
    assert r["rel_l1"] <= rel_l1_max, r
    assert r["flip_frac"] <= flip_max, r
    assert r["p99_rel"] <= P99_TOL, r
    return r
