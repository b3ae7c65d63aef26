"""C ABI checks that need no GPU: the library loads, exports every function
include/tg.h declares, and rejects bad arguments on the host before any
launch."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\**\s+\**(tg_[a-z0-9_]+)\s*\(", src,
                                 flags=re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2604_02586_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtg.so is not built: run __graft_entry__.build()")
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 10, names
    for n in names:
        assert hasattr(L, n), f"{n} declared in tg.h but not exported"


def test_version_status_and_defaults(L):
    from paper_2604_02586_amd import _lib
    assert L.tg_abi_version() == 1
    for k in range(8):
        assert L.tg_status_string(k)
    p = _lib.default_params()
    assert p.alpha_min == np.float32(1 / 255) and p.alpha_max == np.float32(0.99)
    assert p.t_min == np.float32(1e-4) and p.det_min == 1e-12 and p.wsum_min == 1e-3
    assert p.pix_min == 2 and p.views_min == 2 and p.pix_total_min == 3 and p.wsum_total_min == 1e-3
    assert ctypes.sizeof(_lib.Camera) == 80


def _cams(V, W=64, H=48):
    import synth
    from paper_2604_02586_amd import _lib
    return _lib.cameras(synth.ring_cameras(V, 3.0, W, H))


def test_host_side_validation(L):
    from paper_2604_02586_amd import _lib
    p = _lib.default_params()
    cams = _cams(2)
    g = _lib.Gaussians()
    s = _lib.Splats()
    # null buffers
    assert L.tg_preprocess(ctypes.byref(g), 10, cams, 2, ctypes.byref(p), ctypes.byref(s), None) == 1
    # negative sizes
    assert L.tg_preprocess(ctypes.byref(g), -1, cams, 2, ctypes.byref(p), ctypes.byref(s), None) == 1
    # misaligned record array (never dereferenced: rejected on the host)
    fake = ctypes.c_void_p(0x10000)
    g = _lib.Gaussians(fake, fake, fake, fake, None, 0, 0, 0, 0)
    s = _lib.Splats(ctypes.c_void_p(0x10004), fake, fake, fake, None, None)
    assert L.tg_preprocess(ctypes.byref(g), 10, cams, 2, ctypes.byref(p), ctypes.byref(s), None) == 2
    # bad modes
    g.scale_mode = 3
    s.rec = ctypes.c_void_p(0x10000)
    assert L.tg_preprocess(ctypes.byref(g), 10, cams, 2, ctypes.byref(p), ctypes.byref(s), None) == 1
    # accumulator clearing: negative counts, null or misaligned records
    assert L.tg_acc_zero(fake, -1, None) == 1
    assert L.tg_acc_zero(None, 5, None) == 1
    assert L.tg_acc_zero(ctypes.c_void_p(0x10004), 5, None) == 2
    assert L.tg_acc_zero(None, 0, None) == 0
    assert L.tg_acc_zero(fake, 2**62, None) == 1
    # too many views for binning
    big = _cams(33)
    b = _lib.Bins()
    nb = ctypes.c_size_t(0)
    assert L.tg_bin_sort(ctypes.byref(s), 10, big, 33, ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(nb),
                         None) == 7
    # accumulate: views must share one resolution
    mixed = (_lib.Camera * 2)(_cams(1, 64, 48)[0], _cams(1, 32, 32)[0])
    bins = _lib.Bins(fake, fake, fake, fake, fake, 100)
    s2 = _lib.Splats(fake, fake, fake, fake, None, None)
    assert L.tg_splat_accumulate(ctypes.byref(s2), ctypes.byref(bins), 10, mixed, 2, fake, None, ctypes.byref(p),
                                 fake, None, None, None) == 1


def test_batch_accumulate_validation(L):
    from paper_2604_02586_amd import _lib
    p = _lib.default_params()
    cams = _cams(2)
    fake = ctypes.c_void_p(0x10000)
    s = _lib.Splats(fake, fake, fake, fake, None, None)
    b = _lib.Bins(fake, fake, fake, fake, fake, 100)

    def slot(F=1, N=10, V=2, cams_=cams, acc=0x10000):
        sl = _lib.AccSlot(ctypes.addressof(s), ctypes.addressof(b), ctypes.addressof(cams_), N, V, F)
        for f in range(_lib.TG_MAX_FRAMES):
            sl.disp[f] = 0x10000
            sl.acc[f] = acc
        return sl

    arr = (_lib.AccSlot * 9)(*[slot() for _ in range(9)])
    # nothing to do
    assert L.tg_splat_accumulate_batch(arr, 0, ctypes.byref(p), None, None) == 0
    assert L.tg_splat_accumulate_batch(None, 1, ctypes.byref(p), None, None) == 1
    # more slots than one launch takes
    assert L.tg_splat_accumulate_batch(arr, 9, ctypes.byref(p), None, None) == 7
    # frames per slot 1..4
    for F, code in [(0, 7), (5, 7)]:
        one = (_lib.AccSlot * 1)(slot(F=F))
        assert L.tg_splat_accumulate_batch(one, 1, ctypes.byref(p), None, None) == code
    # misaligned accumulators, mixed resolutions, negative sizes
    one = (_lib.AccSlot * 1)(slot(acc=0x10004))
    assert L.tg_splat_accumulate_batch(one, 1, ctypes.byref(p), None, None) == 2
    mixed = (_lib.Camera * 2)(_cams(1, 64, 48)[0], _cams(1, 32, 32)[0])
    one = (_lib.AccSlot * 1)(slot(cams_=mixed))
    assert L.tg_splat_accumulate_batch(one, 1, ctypes.byref(p), None, None) == 1
    one = (_lib.AccSlot * 1)(slot(N=-1))
    assert L.tg_splat_accumulate_batch(one, 1, ctypes.byref(p), None, None) == 1
    # an error in a later slot launches nothing (checked before any launch)
    two = (_lib.AccSlot * 2)(slot(), slot(F=9))
    assert L.tg_splat_accumulate_batch(two, 2, ctypes.byref(p), None, None) == 7


def test_regularize_validation(L):
    from paper_2604_02586_amd import _lib
    p = _lib.default_params()
    assert p.reg_k == 8 and p.static_min_pix == 9 and p.static_frac == 0.9 and p.static_views == 2
    nb = ctypes.c_size_t(0)
    # workspace query needs no buffers
    assert L.tg_regularize(None, None, None, None, 1000, 2, ctypes.byref(p), None, ctypes.byref(nb), None, None,
                           None) == 0
    assert nb.value > 1000 * 150
    fake = ctypes.c_void_p(0x10000)
    g = _lib.Gaussians(fake, fake, fake, fake, None, 0, 0, 0, 0)
    small = ctypes.c_size_t(16)
    assert L.tg_regularize(ctypes.byref(g), ctypes.byref(g), fake, fake, 1000, 2, ctypes.byref(p), fake,
                           ctypes.byref(small), ctypes.byref(g), fake, None) == 3
    big = ctypes.c_size_t(nb.value)
    assert L.tg_regularize(None, ctypes.byref(g), fake, fake, 1000, 2, ctypes.byref(p), fake, ctypes.byref(big),
                           ctypes.byref(g), fake, None) == 1
    glog = _lib.Gaussians(fake, fake, fake, fake, None, 0, 1, 0, 0)
    assert L.tg_regularize(ctypes.byref(glog), ctypes.byref(g), fake, fake, 1000, 2, ctypes.byref(p), fake,
                           ctypes.byref(big), ctypes.byref(g), fake, None) == 7
    p.reg_k = 9
    assert L.tg_regularize(ctypes.byref(g), ctypes.byref(g), fake, fake, 1000, 2, ctypes.byref(p), fake,
                           ctypes.byref(big), ctypes.byref(g), fake, None) == 1


def test_workspace_query_and_cell_counts(L):
    from paper_2604_02586_amd import _lib
    p = _lib.default_params()
    cams = _cams(4, 1920, 1080)
    assert L.tg_num_tiles(cams, 4) == 4 * 120 * 68
    assert L.tg_num_cells(cams, 4, 1000, ctypes.byref(p)) == 4 * 15 * 9
    # rank + bin bits above 32 force a coarser binning
    c_big = L.tg_num_cells(cams, 4, 1 << 26, ctypes.byref(p))
    assert 0 < c_big < 4 * 15 * 9
    s = _lib.Splats()
    b = _lib.Bins()
    b.capacity = 1 << 20
    nb = ctypes.c_size_t(0)
    assert L.tg_bin_sort(ctypes.byref(s), 100000, cams, 4, ctypes.byref(p), ctypes.byref(b), None, ctypes.byref(nb),
                         None) == 0
    assert nb.value >= 4 * (1 << 20) * 2
    small = ctypes.c_size_t(16)
    assert L.tg_bin_sort(ctypes.byref(s), 100000, cams, 4, ctypes.byref(p), ctypes.byref(b), ctypes.c_void_p(0x10000),
                         ctypes.byref(small), None) == 3
    # the allocation-free variant rejects a workspace beyond its scratch on
    # the host, before touching the device
    big = _lib.Bins()
    big.capacity = 1 << 24
    nbig = ctypes.c_size_t(0)
    assert L.tg_bin_sort(ctypes.byref(s), 100000, cams, 4, ctypes.byref(p), ctypes.byref(big), None,
                         ctypes.byref(nbig), None) == 0
    assert nbig.value > _lib.TG_BIN_SORT_STATIC_BYTES
    assert L.tg_bin_sort_static(ctypes.byref(s), 100000, cams, 4, ctypes.byref(p), ctypes.byref(big), None) == 3


def test_product_path_has_no_cpu_fallback():
    """The package imports no oracle code and fails loudly without libtg."""
    import paper_2604_02586_amd
    from paper_2604_02586_amd import _lib
    pkg = os.path.dirname(paper_2604_02586_amd.__file__)
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            txt = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in txt and "from oracle" not in txt, f
    saved = _lib.LIB_PATH, _lib._lib
    try:
        _lib.LIB_PATH, _lib._lib = "/nonexistent/libtg.so", None
        with pytest.raises(ImportError):
            _lib.lib()
    finally:
        _lib.LIB_PATH, _lib._lib = saved
