"""Test helpers: layout conversion between the oracle's path records and the
library's structure-of-arrays path list, and error metrics."""
import numpy as np

KMAX = 4


def oracle_to_soa(p):
    """Oracle PATH_DTYPE records -> dict in the library's SoA layout."""
    import oracle
    return oracle.to_soa(p, KMAX)


def gpu_soa_np(ctx):
    return {k: v.cpu().numpy() for k, v in ctx.paths().items()}


def traced_rows(orc, scene, array, tp):
    """Virtual ray ids of the launched (not point-reflector) rays in hit-list order."""
    per = orc.n_per_src(scene, array, tp)
    ns = orc.n_src(array)
    vps = per + scene.n_pts
    return (np.arange(ns)[:, None] * vps + np.arange(per)[None, :]).reshape(-1)


def rel_err(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_paths_equal(g, o):
    """Bitwise equality of two SoA path dicts."""
    assert len(g["K"]) == len(o["K"]), (len(g["K"]), len(o["K"]))
    for k in ("src", "K", "ray", "tri", "vid", "p", "L", "amp"):
        a, b = np.asarray(g[k]), np.asarray(o[k])
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            raise AssertionError(f"field {k} differs at {bad[:5].tolist()} "
                                 f"(gpu {a[tuple(bad[0])]!r}, oracle {b[tuple(bad[0])]!r})")
