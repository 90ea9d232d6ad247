"""CPU checks of the C ABI: the library loads, exports every declared symbol, and
rejects bad descriptors synchronously (no GPU needed for these paths)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="sdnn.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdnn_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_2004_10908_amd as p
    return p


def test_library_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 12
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    bound = {name for name, _, _ in L.sdnn.PROTOTYPES}
    assert set(names) == bound
    from paper_2004_10908_amd import taskgraph
    tg = declared_functions("sdnn_taskgraph.h")
    assert len(tg) >= 7
    for n in tg:
        assert hasattr(lib, n), n
    assert set(tg) == {name for name, _, _ in taskgraph.PROTOTYPES}


def test_version_and_error_string(L):
    assert "gfx950" in L.sdnn_version()


@pytest.mark.parametrize("kw,status", [
    (dict(k=16), "SDNN_EUNSUPPORTED"), (dict(n_neurons=0), "SDNN_EINVAL"), (dict(n_layers=0), "SDNN_EINVAL"),
    (dict(clamp=0.0), "SDNN_EINVAL"), (dict(clamp=float("inf")), "SDNN_EINVAL"), (dict(max_rows=-1), "SDNN_EINVAL"),
    (dict(flags=0x1, ckpt_every=0), "SDNN_EINVAL"), (dict(flags=0x100), "SDNN_EINVAL"),
    (dict(n_neurons=16), "SDNN_EINVAL"), (dict(n_neurons=65536, flags=0x1, ckpt_every=4), "SDNN_EUNSUPPORTED")])
def test_bad_descriptors_are_rejected(L, kw, status):
    base = dict(n_neurons=1024, n_layers=4, max_rows=100)
    base.update({k: v for k, v in kw.items() if k in base})
    d = L.make_desc(base["n_neurons"], base["n_layers"], base["max_rows"], clamp=kw.get("clamp", 32.0),
                    k=kw.get("k", 32), ckpt_every=kw.get("ckpt_every", 0), flags=kw.get("flags", 0))
    with pytest.raises(L.SdnnError) as e:
        L.sdnn_workspace_size(d)
    assert status in str(e.value)


def test_workspace_and_ckpt_sizes(L):
    d = L.make_desc(4096, 120, 4096, ckpt_every=16, flags=L.sdnn.SDNN_TRAINABLE)
    assert L.sdnn_ckpt_size(d, 4096) == 7 * 4096 * 4096 * 4     # checkpoints Y_16 .. Y_112
    ws = L.sdnn_workspace_size(d)
    assert ws >= (17 + 3) * 4096 * 4096 * 4
    d2 = L.make_desc(4096, 480, 60000)
    assert L.sdnn_ckpt_size(d2, 60000) == 0
    assert L.sdnn_workspace_size(d2) >= 60000 * 4096 * 4


def test_null_arguments_fail_before_any_launch(L):
    lib = L.lib()
    d = L.make_desc(1024, 4, 10)
    h = ctypes.c_void_p()
    st = lib.sdnn_create(ctypes.byref(d), None, None, None, None, 0, None, ctypes.byref(h))
    assert st == L.sdnn.SDNN_EINVAL and not h.value
    assert lib.sdnn_forward(None, None, 0, None, 0, None, None, None, None, None, None) == L.sdnn.SDNN_EINVAL
    assert lib.sdnn_backward(None, None, 0, None, None, None, None, None, None, None, None) == L.sdnn.SDNN_EINVAL
    assert lib.sdnn_set_exec(None, 0) == L.sdnn.SDNN_EINVAL
    lib.sdnn_destroy(None)                         # NULL-safe
    assert lib.sdnn_mse(None, None, -1, None, None, None) == L.sdnn.SDNN_EINVAL


def test_wide_nets_reserve_the_packed_tiles():
    """Forward-only nets the scheduled kernel cannot take keep a second copy of the
    rows (packed tiles of the wide-layer kernels) in the workspace; scheduled and
    trainable nets do not."""
    import paper_2004_10908_amd as L

    def per_row(n, flags=0, ckpt=0):
        a = L.sdnn_workspace_size(L.make_desc(n, 4, 4096, flags=flags, ckpt_every=ckpt))
        b = L.sdnn_workspace_size(L.make_desc(n, 4, 8192, flags=flags, ckpt_every=ckpt))
        return (b - a) / 4096

    assert per_row(16384) >= 2 * 16384 * 4
    assert per_row(6000) >= 2 * 6000 * 4
    assert per_row(4096) < 2 * 4096 * 4
    assert per_row(4096, flags=L.sdnn.SDNN_NO_SCHEDULE) < 2 * 4096 * 4


def test_no_schedule_flag_shrinks_the_workspace():
    """SDNN_NO_SCHEDULE drops the per-layer schedules from the workspace of a net the
    scheduled kernels would otherwise serve."""
    import paper_2004_10908_amd as L
    with_s = L.sdnn_workspace_size(L.make_desc(4096, 8, 1000))
    without = L.sdnn_workspace_size(L.make_desc(4096, 8, 1000, flags=L.sdnn.SDNN_NO_SCHEDULE))
    assert 0 < without < with_s
