"""GPU parity of the background field entering through the box faces (Sec. 2:
packets from diffuse fields such as the UV background) against the oracle,
through the C ABI."""
import numpy as np
import pytest

import parity as PT
from oracle import oracle as O
from paper_1101_4127_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1101_4127_amd import rt
    rt.lib()
    return torch


def bg_case(*, n=20, fp64=True, packets=3000, bg_packets=5000, n_src=3, thin=0.1, ionised=0.9, seed=17):
    w = W.small_mixed(n=n, n_src=n_src, packets=packets, seed=seed, fp64=fp64, ionised_fraction=ionised)
    w = w.with_(cell_cm=w.cell_cm * thin)
    ndot = 0.5 * float(np.sum(w.src_ndot)) if n_src else 1.0e52
    return w.with_(background=W.Background(ndot, w.bins.sed.copy(), bg_packets))


def run_pair(w, *, fp64, steps=1, **tiles):
    from paper_1101_4127_amd import rt
    s = rt.Solve(w, fp64=fp64, **tiles)
    o = O.OracleSolve(w)
    st = [(s.step(seed=w.seed + k), o.step(seed=w.seed + k)) for k in range(steps)]
    f = s.fetch()
    s.release()
    return o, st, f


@pytest.mark.parametrize("n,n_src,bg_packets", [(20, 3, 5000), (13, 0, 4000), (8, 2, 1)])
def test_fp64_matches_oracle(n, n_src, bg_packets):
    w = bg_case(n=n, n_src=n_src, bg_packets=bg_packets, packets=3000 if n_src else 0)
    print(f"background fp64 n={n} sources={n_src} packets={bg_packets}", flush=True)
    o, st, f = run_pair(w, fp64=True, steps=2)
    for g, r in st:
        assert g["packets"] == r["packets"] and g["crossings"] == r["crossings"]
        assert g["n_escaped"] == r["n_escaped"] and g["n_truncated"] == r["n_truncated"]
        assert PT.ledger_close(g, r, 1e-12) <= 1e-12
    PT.compare_state(o, f, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)


def test_fp32_within_stated_tolerance():
    w = bg_case(fp64=False, bg_packets=8000)
    o, st, f = run_pair(w, fp64=False, steps=2)
    for g, r in st:
        assert g["packets"] == r["packets"]
        assert PT.ledger_close(g, r, 1e-5) <= 1e-6
        assert abs(g["crossings"] - r["crossings"]) <= 1e-4 * r["crossings"]
    PT.compare_state(o, f, w, frac_tol=1e-4, temp_tol=1e-4, dep_tol=1e-5)


def test_batches_and_sub_steps():
    """More background packets than records in flight (several batches per
    sub-step), three sub-steps, periodic boundaries and re-emission."""
    w = bg_case(n=12, bg_packets=7001, packets=3000).with_(n_sub=3, periodic=True, path_cells=30,
                                                           dt_s=30.0 * W.MYR_S)
    w = W.with_recombination(w, 0.02)
    o, st, f = run_pair(w, fp64=True, steps=2, inflight=1100)
    for g, r in st:
        assert g["packets"] == r["packets"] and g["crossings"] == r["crossings"]
        assert g["diffuse_packets"] == r["diffuse_packets"]
        assert PT.ledger_close(g, r, 1e-12) <= 1e-12
    assert sum(g["diffuse_packets"] for g, _ in st) > 0
    PT.compare_state(o, f, w, frac_tol=1e-9, temp_tol=1e-9, dep_tol=1e-9)


def test_rejections():
    from paper_1101_4127_amd import rt
    w = bg_case(n=8)
    s = rt.Solve(w.with_(background=None), direct=True)
    with pytest.raises(rt.RTError) as ex:
        rt.rt_set_background(s.h, 1e50, w.bins.sed, 100)
    assert ex.value.status == rt.RT_ESTATE
    s.release()
    s = rt.Solve(w)
    for args in ((-1.0, w.bins.sed, 10), (1e50, np.zeros_like(w.bins.sed), 10), (1e50, w.bins.sed, -1)):
        with pytest.raises(rt.RTError) as ex:
            rt.rt_set_background(s.h, *args)
        assert ex.value.status == rt.RT_EINVAL
    rt.rt_set_background(s.h, 1e50, w.bins.sed, 0)                  # off again
    st = s.step()
    assert st["packets"] == w.packets
    s.release()
    # the fused steps of many solves do not take a background
    wh = W.stromgren_c1(n=8, packets=1000, n_sub=1)
    wh = wh.with_(background=W.Background(1e48, np.ones(1), 100))
    sh = rt.Solve(wh)
    b = rt.Batch(2, wh, fp64=bool(wh.flags & W.FP64_MARCH), max_round_packets=wh.packets,
                 max_tiles=2 * rt.tiles_of(wh.n), graph=False)
    with pytest.raises(rt.RTError) as ex:
        b.step([sh])
    assert ex.value.status == rt.RT_EINVAL
    b.release()
    sh.release()
