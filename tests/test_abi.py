"""The C ABI without a GPU: the library loads, exports every function that
include/rt_mi355x.h declares, its structs match the binding, and argument
checks that precede any device work return RT_EINVAL."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2208_10008_amd as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt_mi355x.h")
PROBE_HEADER = os.path.join(ROOT, "include", "rt_probe.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    assert set(declared_functions()) == set(R.EXPORTS)
    assert set(declared_functions(PROBE_HEADER)) == set(R.PROBE_EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = R.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(declared_functions()) <= exported
    assert set(declared_functions(PROBE_HEADER)) <= exported
    for name in declared_functions(PROBE_HEADER):
        assert hasattr(lib, name), name


def test_library_is_gfx950_code(tmp_path):
    # the offload bundle of the library built here names its target
    sec = tmp_path / "fatbin"
    subprocess.run(["/opt/rocm/llvm/bin/llvm-objcopy", "--dump-section=.hip_fatbin=" + str(sec),
                    R.LIB_PATH, str(tmp_path / "copy.so")], check=True)
    data = sec.read_bytes()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "rt_mi355x.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(rt_split_params), sizeof(rt_hit), sizeof(rt_bvh_info),
         sizeof(rt_node_rec), sizeof(rt_trace_opts));
  printf("%zu %zu %zu %zu %zu %zu\\n", offsetof(rt_node_rec, cost), offsetof(rt_bvh_info, root_lo),
         offsetof(rt_split_params, max_leaf), offsetof(rt_trace_opts, block),
         offsetof(rt_split_params, node_format), offsetof(rt_bvh_info, n_trace_nodes));
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rt_query), offsetof(rt_query, max_bounces),
         offsetof(rt_query, status), offsetof(rt_query, out), offsetof(rt_query, n_hits),
         sizeof(rt_batch_config), offsetof(rt_query, receivers));
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(rt_reception), offsetof(rt_reception, l),
         offsetof(rt_reception, dist), sizeof(rt_receivers), offsetof(rt_receivers, delta),
         offsetof(rt_receivers, cap), offsetof(rt_receivers, count));
  printf("%zu %zu %zu %zu\\n", sizeof(rt_energy), offsetof(rt_energy, k0),
         offsetof(rt_energy, min_power), offsetof(rt_energy, power));
  printf("%zu %zu %zu\\n", sizeof(rt_diffracted), offsetof(rt_diffracted, path),
         offsetof(rt_diffracted, ray8));
  printf("%zu %zu %zu\\n", sizeof(rt_ray_launch), offsetof(rt_ray_launch, first),
         offsetof(rt_ray_launch, n));
  printf("%zu %zu %zu %zu\\n", offsetof(rt_bvh_info, has_stats), offsetof(rt_bvh_info, tree_cost),
         offsetof(rt_bvh_info, root_area), offsetof(rt_bvh_info, leaf_hist));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(rt_trace_opts, cut), offsetof(rt_trace_opts, flags),
         offsetof(rt_trace_opts, chain_ws), offsetof(rt_trace_opts, chain_ws_bytes),
         offsetof(rt_trace_opts, batch_order));
  return 0;
}""")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
                    "-I/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    a, b, c, d, e, g, h, k, m = subprocess.run([str(exe)], capture_output=True, text=True,
                                               check=True).stdout.split("\n")[:9]
    sizes = [int(x) for x in a.split()]
    offs = [int(x) for x in b.split()]
    assert sizes == [ctypes.sizeof(R.rt_split_params), 16, ctypes.sizeof(R.rt_bvh_info),
                     R.NODE_DTYPE.itemsize, ctypes.sizeof(R.rt_trace_opts)]
    assert offs == [R.NODE_DTYPE.fields["cost"][1], R.rt_bvh_info.root_lo.offset,
                    R.rt_split_params.max_leaf.offset, R.rt_trace_opts.block.offset,
                    R.rt_split_params.node_format.offset, R.rt_bvh_info.n_trace_nodes.offset]
    assert [int(x) for x in c.split()] == [ctypes.sizeof(R.rt_query), R.rt_query.max_bounces.offset,
                                           R.rt_query.status.offset, R.rt_query.out.offset,
                                           R.rt_query.n_hits.offset, ctypes.sizeof(R.rt_batch_config),
                                           R.rt_query.receivers.offset]
    assert [int(x) for x in d.split()] == [R.RECEPTION_DTYPE.itemsize, R.RECEPTION_DTYPE.fields["l"][1],
                                           R.RECEPTION_DTYPE.fields["dist"][1],
                                           ctypes.sizeof(R.rt_receivers), R.rt_receivers.delta.offset,
                                           R.rt_receivers.cap.offset, R.rt_receivers.count.offset]
    assert [int(x) for x in e.split()] == [ctypes.sizeof(R.rt_energy), R.rt_energy.k0.offset,
                                           R.rt_energy.min_power.offset, R.rt_energy.power.offset]
    assert [int(x) for x in g.split()] == [R.DIFFRACTED_DTYPE.itemsize,
                                           R.DIFFRACTED_DTYPE.fields["path"][1],
                                           R.DIFFRACTED_DTYPE.fields["ray8"][1]]
    assert [int(x) for x in h.split()] == [R.RAY_LAUNCH_DTYPE.itemsize,
                                           R.RAY_LAUNCH_DTYPE.fields["first"][1],
                                           R.RAY_LAUNCH_DTYPE.fields["n"][1]]
    assert [int(x) for x in k.split()] == [R.rt_bvh_info.has_stats.offset,
                                           R.rt_bvh_info.tree_cost.offset,
                                           R.rt_bvh_info.root_area.offset,
                                           R.rt_bvh_info.leaf_hist.offset]
    assert [int(x) for x in m.split()] == [R.rt_trace_opts.cut.offset,
                                           R.rt_trace_opts.flags.offset,
                                           R.rt_trace_opts.chain_ws.offset,
                                           R.rt_trace_opts.chain_ws_bytes.offset,
                                           R.rt_trace_opts.batch_order.offset]


def test_split_cus_mask_gives_every_xcd_its_share():
    # an MI355X numbers its 256 CUs either by XCD in blocks of 32 or
    # interleaved over its 8 XCDs; the small set must hold k / 8 CUs of every
    # XCD either way (and the large set the rest), so neither stream is ever
    # left without a CU on some XCD
    for k in range(8, 129, 8):
        m = R.rt_split_cus_mask(k)
        cus = [c for c in range(256) if (int(m[c // 32]) >> (c % 32)) & 1]
        assert len(cus) == k
        assert [sum(1 for c in cus if c // 32 == x) for x in range(8)] == [k // 8] * 8
        assert [sum(1 for c in cus if c % 8 == x) for x in range(8)] == [k // 8] * 8
    for k in (0, 4, 12, 136, -8):
        with pytest.raises(R.RtError) as e:
            R.rt_split_cus_mask(k)
        assert e.value.code == R.RT_EINVAL


def test_batch_order_workspace_size():
    # ceil(n / 64) batch keys and 16 class counts per tile of 1024 batches
    assert R.rt_rays_batch_order_ws_bytes(0) == 0
    assert R.rt_rays_batch_order_ws_bytes(1) == 4 * (1 + 16)
    assert R.rt_rays_batch_order_ws_bytes(65536) == 4 * (1024 + 16)
    assert R.rt_rays_batch_order_ws_bytes(65537) == 4 * (1025 + 32)
    assert R.rt_rays_batch_order_ws_bytes(2621442) == 4 * (40961 + 16 * 41)
    assert R.rt_rays_batch_order_ws_bytes(-1) == 0


def test_chain_workspace_size():
    # a 256-byte header (the live-chain count) and one 64-byte chain state per ray
    assert R.rt_trace_chain_ws_bytes(0) == 256
    assert R.rt_trace_chain_ws_bytes(1) == 256 + 64
    assert R.rt_trace_chain_ws_bytes(2621442) == 256 + 64 * 2621442
    assert R.rt_trace_chain_ws_bytes(-1) == 0


def test_defaults():
    lib = R.load()
    p = R.rt_split_params()
    lib.rt_split_params_default(ctypes.byref(p))
    d = R.SplitParams()
    assert (p.alpha, p.t_isect, p.t_trav, list(p.src)) == (d.alpha, d.t_isect, d.t_trav, list(d.src))
    assert (p.max_leaf, p.nbins, p.d_mode, p.d_norm, p.max_depth, p.depth_limit, p.node_format) == \
        (d.max_leaf, d.nbins, 0, 0, d.max_depth, d.depth_limit, 0)


def _build_rc(tris_ptr, n, params):
    lib = R.load()
    h = ctypes.c_void_p()
    return lib.rt_build(tris_ptr, n, ctypes.byref(params), ctypes.byref(h), None), h


@pytest.mark.parametrize("field,value", [("alpha", 1.5), ("alpha", -0.5), ("alpha", float("nan")),
                                         ("max_leaf", 0), ("nbins", 1), ("nbins", 65),
                                         ("d_mode", 4), ("d_norm", 2), ("depth_limit", 0),
                                         ("depth_limit", 65), ("t_isect", 0.0),
                                         ("node_format", 3), ("node_format", -1)])
def test_build_rejects_bad_params(field, value):
    p = R.SplitParams().c()
    setattr(p, field, value)
    host = np.zeros((4, 9), np.float32)   # never read: the checks come first
    rc, h = _build_rc(host.ctypes.data_as(ctypes.c_void_p), 4, p)
    assert rc == R.RT_EINVAL and not h.value
    assert len(R.load().rt_last_error()) > 0


def test_build_rejects_bad_sizes_and_pointers():
    p = R.SplitParams().c()
    host = np.zeros((4, 9), np.float32)
    ptr = host.ctypes.data_as(ctypes.c_void_p)
    assert _build_rc(None, 4, p)[0] == R.RT_EINVAL
    assert _build_rc(ptr, 0, p)[0] == R.RT_EINVAL
    assert _build_rc(ptr, -3, p)[0] == R.RT_EINVAL
    assert _build_rc(ptr, 1 << 30, p)[0] == R.RT_EINVAL
    assert _build_rc(ctypes.c_void_p(host.ctypes.data + 1), 4, p)[0] == R.RT_EINVAL
    q = R.SplitParams(max_leaf=1, depth_limit=3).c()   # 100 facets need 7 halvings
    assert _build_rc(ptr, 100, q)[0] == R.RT_EINVAL
    lib = R.load()
    assert lib.rt_build(ptr, 4, ctypes.byref(p), None, None) == R.RT_EINVAL


def test_null_handles():
    lib = R.load()
    info = R.rt_bvh_info()
    assert lib.rt_bvh_info_get(None, ctypes.byref(info)) == R.RT_EINVAL
    assert lib.rt_bvh_stats(None, ctypes.byref(info)) == R.RT_EINVAL
    host = np.zeros((4, 9), np.float32)
    ptr = host.ctypes.data_as(ctypes.c_void_p)
    assert lib.rt_wedges_noalloc(None, 4, ptr, None) == R.RT_EINVAL
    assert lib.rt_wedges_noalloc(ptr, 0, ptr, None) == R.RT_EINVAL
    assert lib.rt_wedges_noalloc(ptr, 262145, ptr, None) == R.RT_EINVAL   # above its scratch
    assert lib.rt_trace(None, None, 0, None, None) == R.RT_EINVAL
    assert lib.rt_trace_bounces(None, None, 0, 1, None, None, None, None) == R.RT_EINVAL
    assert lib.rt_bvh_download(None, None, 0, None, 0) == R.RT_EINVAL
    assert lib.rt_bvh_export_trace_nodes(None, None, None) == R.RT_EINVAL
    lib.rt_bvh_destroy(None)
    assert lib.rt_rebuild(None, None, 0, None, None) == R.RT_EINVAL
    assert lib.rt_rebuild_async(None, None, 0, None, None) == R.RT_EINVAL
    assert lib.rt_bvh_wait(None) == R.RT_EINVAL


def test_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(R.RtError):
        R.rt_build(torch.zeros((4, 9)), R.SplitParams())


def test_probe_argument_checks():
    lib = R.load()
    buf = np.zeros(64, np.float32)
    p = ctypes.c_void_p(buf.ctypes.data)
    odd = ctypes.c_void_p(buf.ctypes.data + 4)
    assert lib.rt_probe_read(None, 64, 64, 1, 1, p, None) == R.RT_EINVAL
    assert lib.rt_probe_read(p, 64, 64, 1, 1, None, None) == R.RT_EINVAL
    assert lib.rt_probe_read(odd, 64, 64, 1, 1, p, None) == R.RT_EINVAL
    assert lib.rt_probe_read(p, 60, 48, 1, 1, p, None) == R.RT_EINVAL
    assert lib.rt_probe_read(p, 64, 80, 1, 1, p, None) == R.RT_EINVAL    # span > bytes
    assert lib.rt_probe_read(p, 64, 64, 0, 1, p, None) == R.RT_EINVAL
    assert lib.rt_probe_read(p, 64, 64, 1, 0, p, None) == R.RT_EINVAL
    assert lib.rt_probe_copy(None, p, 64, None) == R.RT_EINVAL
    assert lib.rt_probe_copy(p, odd, 64, None) == R.RT_EINVAL
    assert lib.rt_probe_copy(p, p, 64, None) == R.RT_EINVAL          # overlapping ranges
    assert lib.rt_probe_copy(p, ctypes.c_void_p(buf.ctypes.data + 128), 0, None) == R.RT_EINVAL
    assert b"rt_probe" in lib.rt_last_error()


def test_batch_argument_checks():
    """Checks that fail before any device call."""
    lib = R.load()
    h = ctypes.c_void_p()
    assert lib.rt_batch_create(0, ctypes.byref(h)) == R.RT_EINVAL and not h.value
    assert lib.rt_batch_create(65537, ctypes.byref(h)) == R.RT_EINVAL
    assert lib.rt_batch_create(4, None) == R.RT_EINVAL
    q = (R.rt_query * 1)()
    assert lib.rt_batch_set(None, q, 1) == R.RT_EINVAL
    c = R.rt_batch_config(0, 0, 1, 0)
    assert lib.rt_batch_configure(None, ctypes.byref(c)) == R.RT_EINVAL
    assert lib.rt_batch_get_config(None, ctypes.byref(c)) == R.RT_EINVAL
    assert lib.rt_batch_launch(None, None) == R.RT_EINVAL
    assert lib.rt_batch_autotune(None, 1, None, None) == R.RT_EINVAL
    lib.rt_batch_destroy(None)
    assert b"rt_batch" in lib.rt_last_error()


def test_rays_from_directions_argument_checks():
    lib = R.load()
    buf = np.zeros(64, np.float32)
    p = ctypes.c_void_p(buf.ctypes.data)
    assert lib.rt_rays_from_directions(p, 0, 0, 0, 0, 0, 1, p, None) == R.RT_OK   # nothing to do
    assert lib.rt_rays_from_directions(None, 2, 0, 0, 0, 0, 1, p, None) == R.RT_EINVAL
    assert lib.rt_rays_from_directions(p, 2, 0, 0, 0, 0, 1, None, None) == R.RT_EINVAL
    assert lib.rt_rays_from_directions(p, -1, 0, 0, 0, 0, 1, p, None) == R.RT_EINVAL
    assert lib.rt_rays_from_directions(p, 2, 0, 0, 0, 2, 1, p, None) == R.RT_EINVAL
    assert lib.rt_rays_from_directions(p, 2, float("nan"), 0, 0, 0, 1, p, None) == R.RT_EINVAL
    assert lib.rt_rays_from_directions(p, 2, 0, 0, 0, 0, 1, ctypes.c_void_p(buf.ctypes.data + 4),
                                       None) == R.RT_EINVAL


def test_rays_from_directions_many_argument_checks():
    lib = R.load()
    buf = np.zeros(256, np.float32)
    base = buf.ctypes.data
    base += (-base) % 16
    p = ctypes.c_void_p(base)
    f = lib.rt_rays_from_directions_many
    assert f(p, 4, p, 0, 0, 1, p, 2, None) == R.RT_OK                 # no launch: nothing to do
    assert f(p, 4, p, 1, 0, 1, p, 0, None) == R.RT_OK                 # no rows
    assert f(None, 4, p, 1, 0, 1, p, 2, None) == R.RT_EINVAL
    assert f(p, 4, None, 1, 0, 1, p, 2, None) == R.RT_EINVAL
    assert f(p, 4, p, 1, 0, 1, None, 2, None) == R.RT_EINVAL
    assert f(p, 4, p, -1, 0, 1, p, 2, None) == R.RT_EINVAL
    assert f(p, 4, p, 1, 0, 1, p, -2, None) == R.RT_EINVAL
    assert f(p, -4, p, 1, 0, 1, p, 2, None) == R.RT_EINVAL
    assert f(p, 4, p, 1, 2, 1, p, 2, None) == R.RT_EINVAL             # tmin > tmax
    assert f(p, 4, p, 1, float("nan"), 1, p, 2, None) == R.RT_EINVAL
    assert f(p, 4, ctypes.c_void_p(base + 8), 1, 0, 1, p, 2, None) == R.RT_EINVAL
    assert f(p, 4, p, 1, 0, 1, ctypes.c_void_p(base + 4), 2, None) == R.RT_EINVAL
    assert R.RAY_LAUNCH_DTYPE.itemsize == 32


def test_reception_argument_checks():
    """Checks that fail before any device call."""
    lib = R.load()
    buf = np.zeros(256, np.float64)
    base = buf.ctypes.data
    base += (-base) % 256
    p = ctypes.c_void_p(base)

    def rx(**kw):
        r = R.rt_receivers(pos=base, n=2, reserved=0, delta=0.01, rec=base + 256, cap=4,
                           count=base + 512)
        for k, v in kw.items():
            setattr(r, k, v)
        return ctypes.byref(r)

    seg = lib.rt_receive_segments
    assert seg(p, p, 4, 2, None, None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(n=-1), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(reserved=1), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(pos=None), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(pos=base + 4), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(delta=float("nan")), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(delta=-1.0), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(cap=-1), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(cap=1 << 31), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(rec=None), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(rec=base + 8), None) == R.RT_EINVAL
    assert seg(p, p, 4, 2, rx(count=None), None) == R.RT_EINVAL
    # field points are read as constant data: nothing the call writes may overlap them
    for kw in (dict(rec=base), dict(rec=base + 32), dict(count=base + 40), dict(pos=base + 512)):
        assert seg(p, p, 4, 2, rx(**kw), None) == R.RT_EINVAL, kw
        assert b"overlaps" in lib.rt_last_error(), kw
    assert lib.rt_trace_receive(None, p, 4, 2, p, None, None, rx(), None) == R.RT_EINVAL
    assert seg(p, p, 4, 0, rx(), None) == R.RT_EINVAL                 # max_bounces
    assert seg(p, p, 4, 65, rx(), None) == R.RT_EINVAL
    assert seg(p, p, -1, 2, rx(), None) == R.RT_EINVAL
    assert seg(p, p, 1 << 31, 2, rx(), None) == R.RT_EINVAL
    assert seg(None, p, 4, 2, rx(), None) == R.RT_EINVAL
    assert seg(ctypes.c_void_p(base + 4), p, 4, 2, rx(), None) == R.RT_EINVAL
    assert lib.rt_trace_receive(None, p, 4, 2, p, None, None, rx(), None) == R.RT_EINVAL
    ws = lib.rt_receive_dedup_workspace
    assert ws(10, 3) == 256 and ws(100, 0) == 512 and ws(-1, 0) == -1 and ws(1 << 31, 0) == -1
    assert ws(0, -1) == -1
    assert lib.rt_receive_dedup(p, 4, 2, rx(), None, 1 << 20, None) == R.RT_EINVAL
    assert lib.rt_receive_dedup(p, 4, 2, rx(), ctypes.c_void_p(base + 8), 1 << 20, None) == R.RT_EINVAL
    assert lib.rt_receive_dedup(p, 4, 2, rx(), p, 8, None) == R.RT_EINVAL   # too small
    assert lib.rt_receive_dedup(p, 4, 0, rx(), p, 1 << 20, None) == R.RT_EINVAL
    assert lib.rt_receive_dedup(p, 4, 2, rx(cap=0), None, 0, None) == R.RT_OK   # nothing stored


def test_energy_argument_checks():
    """Checks that fail before any device call: the energy struct is checked
    first, then the tree handle."""
    lib = R.load()
    buf = np.zeros(64, np.float64)
    base = buf.ctypes.data + (-buf.ctypes.data) % 64
    p = ctypes.c_void_p(base)

    def en(**kw):
        e = R.rt_energy(material=base, refl=base, n_materials=2, reserved=0, k0=1e-4,
                        min_power=1e-9, power=None)
        for k, v in kw.items():
            setattr(e, k, v)
        return ctypes.byref(e)

    f = lib.rt_trace_energy
    for kw, word in ((dict(material=None), b"material"), (dict(material=base + 2), b"material"),
                     (dict(n_materials=-1), b"n_materials"), (dict(reserved=3), b"reserved"),
                     (dict(refl=None), b"refl"), (dict(refl=base + 4), b"refl"),
                     (dict(k0=0.0), b"k0"), (dict(k0=float("inf")), b"k0"),
                     (dict(min_power=-1.0), b"min_power"), (dict(min_power=float("nan")), b"min_power"),
                     (dict(power=base + 4), b"power")):
        assert f(None, p, 4, 2, en(**kw), p, None, None, None, None) == R.RT_EINVAL, kw
        assert word in lib.rt_last_error(), (kw, lib.rt_last_error())
    assert f(None, p, 4, 2, None, p, None, None, None, None) == R.RT_EINVAL
    # a valid struct (refl may be NULL without materials) reaches the tree check
    assert f(None, p, 4, 2, en(refl=None, n_materials=0), p, None, None, None, None) == R.RT_EINVAL
    assert b"tree" in lib.rt_last_error()


def test_diffraction_argument_checks():
    """Checks that fail before any device call."""
    lib = R.load()
    buf = np.zeros(64, np.float64)
    base = buf.ctypes.data + (-buf.ctypes.data) % 64
    p = ctypes.c_void_p(base)
    odd = ctypes.c_void_p(base + 2)
    w = lib.rt_wedges
    assert w(None, 4, p, None) == R.RT_EINVAL
    assert w(p, 4, None, None) == R.RT_EINVAL
    assert w(odd, 4, p, None) == R.RT_EINVAL
    assert w(p, 0, p, None) == R.RT_EINVAL and w(p, 1 << 29, p, None) == R.RT_EINVAL
    d = lib.rt_diffract_segments

    def call(**kw):
        a = dict(tris=p, n_tris=4, nbr=p, seg=p, hits=p, n=4, nb=2, delta=0.01, cone=p, n_cone=4,
                 out=p, cap=4, count=p)
        a.update(kw)
        return d(a["tris"], a["n_tris"], a["nbr"], a["seg"], a["hits"], a["n"], a["nb"], a["delta"],
                 a["cone"], a["n_cone"], a["out"], a["cap"], a["count"], None)

    for kw in (dict(tris=None), dict(nbr=None), dict(count=None), dict(count=odd), dict(n_tris=0),
               dict(n=-1), dict(n=1 << 31), dict(nb=0), dict(nb=65), dict(delta=-1.0),
               dict(delta=float("inf")), dict(n_cone=-1), dict(n_cone=1025), dict(cone=None),
               dict(cap=-1), dict(cap=1 << 31), dict(out=None), dict(seg=None), dict(hits=odd)):
        assert call(**kw) == R.RT_EINVAL, kw
