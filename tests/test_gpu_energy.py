"""Energy stop rule (Sec. III-B) on the GPU through the C ABI.

* min_power = 0 never stops a chain: results equal rt_trace_bounces bit for
  bit in every node format.
* Against the CPU checker's float64 chains with the same rule: on chains
  that agree with the checker's hit for hit (same facets, distances within
  1e-5, clean margins), the stop point must be the checker's except where the
  checker's power at either stop lies within 1e-4 of the threshold (a float32
  segment's path length is within about 1e-5 of the float64 one, and P goes
  with 1 / l^2); the last hit's power agrees within 1e-4.
* With field points, the receptions are exactly those of the fixed-order
  chains on the segments the energy rule launched.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import icosphere, scenes, workloads

from _parity import keyed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
NTHREADS = min(16, os.cpu_count() or 1)
K0 = workloads.free_space_k0()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.load()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def city():
    tris, half = workloads.multiscene_scene(1)
    src = scenes.free_point(np.random.default_rng(3), half * 0.3, tris, 25.0)
    return tris, half, src, workloads.city_materials(tris.shape[0], 1)


def energy(material, thr, n):
    return R.Energy(dev(material), dev(workloads.REFLECTION), K0, thr,
                    power=torch.full((n,), -1.0, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("fmt", ["bin2", "f4", "q4"])
def test_zero_threshold_equals_fixed_order(city, fmt):
    tris, _, src, mat = city
    rays = dev(workloads.multiscene_rays(src, 6))
    bvh = R.BVH(dev(tris), R.SplitParams(alpha=0.4, src=src, node_format=fmt))
    e = energy(mat, 0.0, rays.shape[0])
    out, pl, nh = bvh.trace_energy(rays, 6, e)
    out2, pl2, nh2 = bvh.trace_bounces(rays, 6)
    assert torch.equal(out, out2) and torch.equal(pl, pl2) and torch.equal(nh, nh2)
    pw = e.power.cpu().numpy()
    hn = nh.cpu().numpy()
    assert np.all(pw[hn == 0] == 0) and np.all(pw[hn > 0] > 0)


def stop_agreement(tris, rays, mat, thr, nb, params, out_e, nh, pw, out_f):
    """out_e / nh / pw: the GPU's energy chains; out_f: its fixed-order chains."""
    tree = oracle.build_tree(tris, params)
    ch, opw = oracle.bounces_energy(tris, rays, nb, mat, workloads.REFLECTION, K0, thr, tree=tree,
                                    nthreads=NTHREADS, segments=False)
    fixed = oracle.bounces(tris, rays, nb, tree=tree, nthreads=NTHREADS, segments=False)
    m = rays.shape[0]
    # the GPU's energy chain is a prefix of its fixed-order chain
    for b in range(nb):
        pre = b < nh
        assert np.array_equal(out_e[b][pre], out_f[b][pre]), f"segment {b}"
        assert np.all(out_e[b][~pre, 0] == -1)
    ids_f = out_f[..., 0]
    t_f = out_f[..., 1].view(np.float32).astype(np.float64)
    # the checker's power after each hit of its fixed-order chain (reflection keeps |d|)
    dn = np.sqrt((rays[:, 4:7].astype(np.float64) ** 2).sum(1))
    path, gain = np.zeros(m), np.ones(m)
    Pb = np.full((nb, m), np.nan)
    for b in range(nb):
        hit = fixed.id[b] >= 0
        path = path + np.where(hit, fixed.t[b], 0.0) * dn
        gain = gain * np.where(hit, workloads.REFLECTION[mat[np.where(hit, fixed.id[b], 0)]], 1.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            Pb[b] = np.where(hit, gain * K0 / (path * path), np.nan)
    # chains that agree with the checker's on every hit either stop can reach
    agree = np.ones(m, bool)
    reach = np.maximum(ch.n_hits, nh)
    for b in range(nb):
        live = b < reach
        same = (ids_f[b] == fixed.id[b]) & (fixed.margin[b] > 1e-4)
        with np.errstate(invalid="ignore"):
            tclose = (fixed.id[b] < 0) | (np.abs(t_f[b] - fixed.t[b]) <= 1e-5 * np.maximum(fixed.t[b], 1e-3))
        agree &= ~live | (same & tclose)
    differ = agree & (nh != ch.n_hits)
    border = np.zeros(m, bool)
    for k in np.nonzero(differ)[0]:
        border[k] = any(abs(Pb[h - 1, k] / thr - 1) <= 1e-4 for h in (nh[k], ch.n_hits[k]) if 0 < h <= nb)
    bad = differ & ~border
    assert not bad.any(), f"{bad.sum()} chains stop at another hit away from the threshold, e.g. {np.nonzero(bad)[0][:5]}"
    eq = agree & (nh == ch.n_hits) & (nh > 0)
    rel = np.abs(pw[eq] - opw[eq]) / opw[eq]
    assert rel.size and rel.max() <= 1e-4, rel.max()
    stopped = (opw < thr) & (ch.n_hits > 0)
    return {"rays": m, "agree": int(agree.sum()), "stop_differs": int(differ.sum()),
            "stopped_by_energy": float(stopped.mean()), "power_rel_max": float(rel.max())}


def test_city_energy_against_the_checker(city):
    tris, _, src, mat = city
    rays = workloads.multiscene_rays(src, 6)
    thr, nb = 1e-10, 6
    bvh = R.BVH(dev(tris), R.SplitParams(alpha=0.4, src=src))
    e = energy(mat, thr, rays.shape[0])
    out, pl, nh = bvh.trace_energy(dev(rays), nb, e)
    out_f, _, _ = bvh.trace_bounces(dev(rays), nb)
    st = stop_agreement(tris, rays, mat, thr, nb, oracle.SplitParams(alpha=0.4, src=src),
                        out.cpu().numpy(), nh.cpu().numpy(), e.power.cpu().numpy(),
                        out_f.cpu().numpy())
    log("city energy:", st)
    assert st["agree"] > 0.98 * st["rays"] and st["stopped_by_energy"] > 0.1


@pytest.mark.parametrize("fmt", ["bin2", "q4"])
def test_indoor_energy_against_the_checker(fmt):
    w = workloads.paper_indoor()
    rays = w.rays(6)
    thr, nb = 1e-7, 6
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf,
                                           node_format=fmt))
    e = energy(w.material, thr, rays.shape[0])
    out, pl, nh = bvh.trace_energy(dev(rays), nb, e)
    out_f, _, _ = bvh.trace_bounces(dev(rays), nb)
    st = stop_agreement(w.tris, rays, w.material, thr, nb,
                        oracle.SplitParams(alpha=w.alpha, src=w.tx, max_leaf=w.max_leaf),
                        out.cpu().numpy(), nh.cpu().numpy(), e.power.cpu().numpy(),
                        out_f.cpu().numpy())
    log(f"indoor energy ({fmt}):", st)
    assert st["agree"] > 0.95 * st["rays"] and st["stopped_by_energy"] > 0.9


def test_energy_receptions_are_those_of_the_launched_segments(city):
    tris, half, src, mat = city
    lv, nb, thr = 6, 6, 1e-10
    rays = dev(workloads.multiscene_rays(src, lv))
    n = rays.shape[0]
    rx = dev(workloads.field_points(tris, half * 0.5, 32, 5))
    delta = float(icosphere.edge_angles(lv).mean())
    bvh = R.BVH(dev(tris), R.SplitParams(alpha=0.4, src=src))
    e = energy(mat, thr, n)
    ra = R.Receivers(rx, delta, 1 << 16)
    out, pl, nh = bvh.trace_energy(rays, nb, e, receivers=ra)
    rb = R.Receivers(rx, delta, 1 << 16)
    bvh.trace_receive(rays, nb, rb)
    hn, pw = nh.cpu().numpy(), e.power.cpu().numpy()
    # segments launched: after an energy stop the hit count, else one more (up to nb)
    launched = np.where((hn > 0) & (pw < thr), hn, np.minimum(hn + 1, nb))
    a = ra.records()
    b = rb.records()
    b = b[b["order"] < launched[b["ray"]]]
    (ka, kka), (kb, kkb) = keyed(a), keyed(b)
    assert kka == kkb and np.array_equal(ka["l"], kb["l"]) and np.array_equal(ka["dist"], kb["dist"])
    log(f"energy receptions: {a.size} of {rb.count()} fixed-order receptions")
    assert 0 < a.size < rb.count()


def test_energy_edge_cases(city):
    tris, _, src, mat = city
    bvh = R.BVH(dev(tris), R.SplitParams(alpha=0.4, src=src))
    # empty ray set
    e = energy(mat, 1e-10, 0)
    out, pl, nh = bvh.trace_energy(torch.empty((0, 8), dtype=torch.float32, device="cuda"), 4, e)
    assert out.shape == (4, 0, 4)
    # unknown materials reflect nothing: every chain stops at its first hit, as in the checker
    rays = workloads.multiscene_rays(src, 4)
    bad = np.full(tris.shape[0], 7, np.int32)
    e = energy(bad, 1e-30, rays.shape[0])
    out, pl, nh = bvh.trace_energy(dev(rays), 4, e)
    hn = nh.cpu().numpy()
    ch, pw = oracle.bounces_energy(tris, rays, 4, bad, workloads.REFLECTION, K0, 1e-30, nthreads=NTHREADS)
    assert hn.max() == 1 and np.array_equal(hn, ch.n_hits)
    assert np.all(e.power.cpu().numpy() == 0.0)


@pytest.mark.slow
def test_city24k_full_size_energy():
    """The benchmark's launch (city24k, level 9, 6 segments) at the 1e-10
    threshold: 20,000 sampled chains stop where the checker's stop."""
    w = workloads.city24k()
    mat = workloads.city_materials(w.n_tris, 0)
    thr, nb = 1e-10, w.max_bounces
    bvh = R.BVH(dev(w.tris), R.SplitParams(alpha=0.4, src=w.tx))
    e = energy(mat, thr, w.n_rays)
    d_rays = dev(w.rays)
    out, _, nh = bvh.trace_energy(d_rays, nb, e)
    out_f, _, _ = bvh.trace_bounces(d_rays, nb)
    rng = np.random.default_rng(13)
    pick = np.sort(rng.choice(w.n_rays, 20_000, replace=False))
    st = stop_agreement(w.tris, w.rays[pick], mat, thr, nb, oracle.SplitParams(alpha=0.4, src=w.tx),
                        out.cpu().numpy()[:, pick], nh.cpu().numpy()[pick],
                        e.power.cpu().numpy()[pick], out_f.cpu().numpy()[:, pick])
    log("city24k energy (sampled):", st)
    assert st["agree"] > 0.98 * st["rays"] and st["stopped_by_energy"] > 0.05
