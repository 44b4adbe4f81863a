"""Comparison helpers shared by the GPU parity tests."""
import numpy as np

LUM = np.array([0.2126, 0.7152, 0.0722])


def rel_err(a, b, floor=1e-3):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.abs(a - b) / (np.abs(b) + floor)


def tags(rec):
    return np.asarray(rec[:, 12]).astype(np.uint64).astype(np.uint32)


def compare_reservoirs(gpu, ref, active=None, tol_mean=1e-4, tol_flip=1e-3, label=""):
    """Element-wise comparison of reservoir records (oracle layout).  Pixels
    whose selected-sample tag differs are counted as flips; the others must
    agree in every field."""
    n = len(ref)
    act = np.ones(n, bool) if active is None else active
    tg, tr = tags(gpu), tags(ref)
    same = (tg == tr) & act
    flips = np.mean(tg[act] != tr[act]) if act.any() else 0.0
    out = {"flips": float(flips), "count": int(act.sum())}
    # integer fields exact on unflipped pixels
    assert np.array_equal(gpu[same, 11], ref[same, 11]), f"{label} M differs"
    assert np.array_equal(gpu[same, 13], ref[same, 13]), f"{label} prim differs"
    nonempty = same & (ref[:, 10] > 0)
    for name, cols, floor in (("y", slice(0, 3), 1e-3), ("n", slice(3, 6), 1e-3),
                              ("L", slice(6, 9), 1e-3), ("wsum", slice(9, 10), 1e-6),
                              ("W", slice(10, 11), 1e-6)):
        sel = nonempty if name in ("y", "n", "L", "W") else same
        if not sel.any():
            continue
        e = rel_err(gpu[sel, cols], ref[sel, cols], floor)
        out[name] = float(e.mean())
        out[name + "_max"] = float(e.max())
    # W = 0 exactly where the oracle has W = 0 (up to flips)
    zero_mismatch = same & ((gpu[:, 10] > 0) != (ref[:, 10] > 0))
    out["zeroW_mismatch"] = float(zero_mismatch.mean())
    assert flips <= tol_flip, f"{label} flips {flips:.2e} > {tol_flip:g} ({out})"
    for name in ("y", "n", "L", "wsum", "W"):
        if name in out:
            assert out[name] <= tol_mean, f"{label} {name} mean rel err {out[name]:.2e} ({out})"
    assert out["zeroW_mismatch"] <= tol_flip, f"{label} W=0 mismatch ({out})"
    return out, same


def compare_images(gpu, ref, same, tol=1e-4, label=""):
    """Mean relative error over unflipped pixels (per channel, Sec. 4 MAPE style
    with floor 0.01)."""
    e = np.abs(gpu[same] - ref[same]) / (np.abs(ref[same]) + 1e-2)
    m = float(e.mean())
    assert m <= tol, f"{label} mean rel image err {m:.2e} > {tol:g}"
    return m
