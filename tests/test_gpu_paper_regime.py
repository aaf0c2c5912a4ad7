"""The paper's own regime (Sec. IV): paper-size stand-in scenes (study room,
2,778 facets, 250 per leaf, alpha 0.7, reflection order <= 2; campus, 7,608
facets, 820 per leaf, alpha 0.4, order <= 3), on the GPU through the C ABI:

* the traditional (alpha = 1) and proposed trees equal the checker's node
  for node at these leaf sizes;
* every traced segment at icosphere level 6 is re-traced by the checker from
  the GPU's own segment ray (rule of tests/_parity.py);
* the paths received at the paper's Rx are the same with both trees (the
  paper's Figs. 10-11: acceleration removes only useless tests), and agree
  with receptions on the checker's float64 chains.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2208_10008_amd as R
from rtgen import icosphere, workloads

from _parity import agree_with_checker, canonical_compare, compare_hits, keyed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
NTHREADS = min(16, os.cpu_count() or 1)


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


SCENES = {"indoor": workloads.paper_indoor, "outdoor": workloads.paper_outdoor}


@pytest.fixture(scope="module", params=sorted(SCENES))
def scene(request):
    return SCENES[request.param]()


def params(w, alpha, fmt="bin2"):
    return (R.SplitParams(alpha=alpha, src=w.tx, max_leaf=w.max_leaf, node_format=fmt),
            oracle.SplitParams(alpha=alpha, src=w.tx, max_leaf=w.max_leaf))


@pytest.mark.parametrize("kind", ["traditional", "proposed"])
def test_paper_trees_equal_the_checker(scene, kind):
    alpha = 1.0 if kind == "traditional" else scene.alpha
    gp, op = params(scene, alpha)
    bvh = R.BVH(dev(scene.tris), gp)
    nodes, perm = bvh.download()
    tree = oracle.build_tree(scene.tris, op)
    canonical_compare(nodes, perm, tree)
    log(f"{scene.name} {kind}: {tree.n_nodes} nodes, depth {bvh.info().depth}")


@pytest.mark.parametrize("fmt", ["bin2", "q4"])
def test_paper_every_segment_against_the_checker(scene, fmt):
    gp, op = params(scene, scene.alpha, fmt)
    bvh = R.BVH(dev(scene.tris), gp)
    rays = scene.rays(6)
    n, nb = rays.shape[0], scene.max_bounces
    seg = torch.empty((nb, n, 8), dtype=torch.float32, device="cuda")
    out, _, nh = bvh.trace_bounces(dev(rays), nb, seg_rays=seg)
    o = out.cpu().numpy()
    ids, t = o[..., 0], o[..., 1].view(np.float32).astype(np.float64)
    seg_np = seg.cpu().numpy()
    tree = oracle.build_tree(scene.tris, op)
    live = np.ones(n, bool)
    prev = np.full(n, -1, np.int32)
    total = 0
    for b in range(nb):
        idx = np.nonzero(live)[0]
        if idx.size == 0:
            break
        rb = seg_np[b, idx]
        ref = oracle.trace_bvh(tree, rb, skip=prev[idx], nthreads=NTHREADS)
        compare_hits(scene.tris, rb, ids[b, idx], t[b, idx], ref, skip=prev[idx])
        total += idx.size
        prev[idx] = ids[b, idx]
        live[idx[ids[b, idx] < 0]] = False
    assert np.array_equal(nh.cpu().numpy(), (ids >= 0).sum(0))
    log(f"{scene.name} {fmt}: {total} segments checked")


def test_paper_paths_do_not_depend_on_the_split(scene):
    lv = 7
    rays = dev(scene.rays(lv))
    n, nb = rays.shape[0], scene.max_bounces
    delta = float(icosphere.edge_angles(lv).mean())
    res = {}
    for kind, alpha in (("traditional", 1.0), ("proposed", scene.alpha)):
        bvh = R.BVH(dev(scene.tris), params(scene, alpha)[0])
        recv = R.Receivers(torch.tensor([scene.rx], dtype=torch.float64, device="cuda"), delta, 1 << 16)
        out, pl, nh = bvh.trace_receive(rays, nb, recv)
        recv.dedup(out, nb)
        res[kind] = (out.cpu().numpy(), recv.records())
    (oa, ra), (ob, rb) = res["traditional"], res["proposed"]
    same_chain = np.all(oa[..., 0] == ob[..., 0], axis=0) & np.all(oa[..., 1] == ob[..., 1], axis=0)
    log(f"{scene.name}: chains identical on {same_chain.mean() * 100:.4f} % of {n} rays")
    assert same_chain.mean() > 0.999
    ka, kb = keyed(ra[same_chain[ra["ray"]]]), keyed(rb[same_chain[rb["ray"]]])
    assert ka[1] == kb[1]
    assert np.array_equal(ka[0]["l"], kb[0]["l"]) and np.array_equal(ka[0]["keep"], kb[0]["keep"])
    kept = ka[0][ka[0]["keep"] == 1]
    log(f"{scene.name}: {ka[0].size} receptions, {kept.size} paths, by order "
        f"{np.bincount(kept['order'], minlength=nb).tolist()}")
    assert kept.size >= 3 and np.any(kept["order"] == 0)     # the direct path at least


def test_paper_receptions_against_float64_chains(scene):
    lv = 6
    rays = scene.rays(lv)
    nb = scene.max_bounces
    delta = float(icosphere.edge_angles(lv).mean())
    gp, op = params(scene, scene.alpha)
    bvh = R.BVH(dev(scene.tris), gp)
    rx = np.array([scene.rx], np.float64)
    recv = R.Receivers(dev(rx), delta, 1 << 16)
    out, _, _ = bvh.trace_receive(dev(rays), nb, recv)
    o = out.cpu().numpy()
    st = agree_with_checker(scene.tris, rays, rx, delta, nb, op, recv.records(), o[..., 0],
                            o[..., 1].view(np.float32).astype(np.float64), nthreads=NTHREADS)
    log(f"{scene.name} receptions vs float64 chains: {st}")
    assert st["compared"] >= 0.9 * st["checker"] and st["checker"] > 0
