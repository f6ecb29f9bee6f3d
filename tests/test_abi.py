"""CPU checks of the boundary: the HIP library loads, exports every symbol
declared in include/dmgs.h, and its pure host logic (defaults, footprint,
option validation) behaves as documented.  No GPU call is made."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "dmgs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmgs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_2608_00760_amd import _abi, _build
    if not os.path.exists(_abi.LIB_PATH):
        _build.build(force=False)
    _abi.lib()
    return _abi


def test_every_declared_symbol_is_exported(abi):
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(abi.lib(), n), n
    assert sorted(abi.SIGNATURES) == names


def test_default_options_and_footprint(abi):
    o = abi.default_options(256)
    assert tuple(o.n) == (256, 256, 256) and o.nu_pre == 2 and o.nu_post == 2 and o.rtol == 1e-10
    lib = abi.lib()
    b64 = lib.dmgs_workspace_bytes(C.byref(o))
    nv = 257 ** 3
    assert b64 >= 4 * nv * 8            # D, mu, scratch, defect on the finest level
    o.precision = abi.DMGS_FP32_IN_FP64
    b32 = lib.dmgs_workspace_bytes(C.byref(o))
    assert b32 > b64 - nv * 8
    for bad in (5, 20, 1, 0, 2048):
        ob = abi.default_options(bad)
        assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0, bad
    # general grids (different counts or spacings per axis): valid when every
    # axis halves down to a smallest count of 2 or 3, float64 RB-GS only
    ob = abi.default_options(64)
    ob.n[2] = 32
    assert lib.dmgs_workspace_bytes(C.byref(ob)) > 0
    for n3, ok in (((128, 64, 64), True), ((96, 64, 48), True), ((10, 8, 8), False), ((64, 64, 1), False),
                   ((512, 16, 16), True), ((1024, 16, 16), False), ((2048, 1024, 1024), False)):
        ob = abi.default_options(8)
        ob.n[0], ob.n[1], ob.n[2] = n3
        assert (lib.dmgs_workspace_bytes(C.byref(ob)) > 0) == ok, n3
    ob = abi.default_options(128)
    ob.n[1] = ob.n[2] = 64
    ob.precision = abi.DMGS_FP32_IN_FP64
    assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0
    ob = abi.default_options(64)
    ob.h_axis[0], ob.h_axis[1], ob.h_axis[2] = 1.0, 2.0, 1.0   # unequal spacing alone makes a general grid
    assert lib.dmgs_workspace_bytes(C.byref(ob)) > 0
    ob.precision = abi.DMGS_FP32_IN_FP64
    assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0
    ob.h_axis[1] = 1.0                                          # equal spacings: a cubic plan again
    assert lib.dmgs_workspace_bytes(C.byref(ob)) > 0
    ob.h_axis[1] = -1.0
    assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0
    ob = abi.default_options(64)
    ob.nu_pre = ob.nu_post = 0
    assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0
    for good in (2, 3, 6, 96, 192, 512):
        assert lib.dmgs_workspace_bytes(C.byref(abi.default_options(good))) > 0
    # a plan that has run dmgs_forward_vjp also holds a second work set
    for prec in (abi.DMGS_FP64, abi.DMGS_FP32_IN_FP64):
        o = abi.default_options(256)
        o.precision = prec
        base, both = lib.dmgs_workspace_bytes(C.byref(o)), lib.dmgs_forward_vjp_workspace_bytes(C.byref(o))
        assert base + nv * 8 <= both < 2 * base
    assert lib.dmgs_forward_vjp_workspace_bytes(C.byref(abi.default_options(20))) == 0


def test_padded_finest_level_footprint(abi, monkeypatch):
    """Refinement plans whose finest-level passes all take a row pitch pad
    that level's float32 rows to a multiple of four elements (n = 257: 260):
    its seven float32 arrays (D, mu, w, iterate, right-hand side, partner,
    defect) grow by n^2 (py - n) elements each, and the second work set of
    dmgs_forward_vjp (iterate, right-hand side, partner, defect) likewise.
    Odd smoothing counts, weighted Jacobi, float64 plans, levels the block
    passes take and DMGS_PAD=0 keep the dense layout."""
    lib = abi.lib()

    def both(o):
        return lib.dmgs_workspace_bytes(C.byref(o)), lib.dmgs_forward_vjp_workspace_bytes(C.byref(o))

    for N, py in ((256, 260), (128, 132), (96, 100)):
        o = abi.default_options(N)
        o.precision = abi.DMGS_FP32_IN_FP64
        n = N + 1
        monkeypatch.setenv("DMGS_PAD", "0")
        dense = both(o)
        monkeypatch.delenv("DMGS_PAD")
        padded = both(o)
        grow = n * n * (py - n) * 4
        assert padded[0] - dense[0] == 7 * grow, N
        assert padded[1] - dense[1] == 11 * grow, N
    for change in ({"nu_pre": 1, "nu_post": 1}, {"nu_post": 3}, {"smoother": abi.DMGS_WJACOBI},
                   {"precision": abi.DMGS_FP64}, {"n": 64}):
        o = abi.default_options(change.pop("n", 256))
        o.precision = abi.DMGS_FP32_IN_FP64
        for k, v in change.items():
            setattr(o, k, v)
        monkeypatch.setenv("DMGS_PAD", "0")
        dense = both(o)
        monkeypatch.delenv("DMGS_PAD")
        assert both(o) == dense, change


def test_options_layout_matches_the_header(abi):
    """dmgs_default_options clears sizeof(dmgs_options) bytes and then sets the
    defaults; in a buffer pre-filled with a sentinel, it writes up to the last
    byte of the binding's struct (the zero high bytes of `ndim` = 3) and no
    further."""
    size = C.sizeof(abi.Options)
    buf = (C.c_uint8 * (size + 64))(*([0xAB] * (size + 64)))
    abi.lib().dmgs_default_options(32, C.cast(buf, C.POINTER(abi.Options)))
    written = [i for i in range(size + 64) if buf[i] != 0xAB]
    assert written[-1] + 1 <= size and all(buf[i] == 0 for i in range(written[-1] + 1, size))
    assert buf[size] == 0xAB
    o = abi.Options.from_buffer(buf)
    assert o.adjoint_schedule == 0 and o.ir_adaptive == 1 and o.ir_inner_cycles == 8 and o.ndim == 3
    o.adjoint_schedule = 2
    assert abi.lib().dmgs_workspace_bytes(C.byref(o)) == 0


def test_two_dimensional_options(abi):
    lib = abi.lib()
    o = abi.default_options(8192)
    o.ndim = 2
    b = lib.dmgs_workspace_bytes(C.byref(o))
    # per level D, mu, partner; below the finest u and q; above the coarsest
    # the written defect; one float64 scratch field of the finest size; and
    # under 1 MiB of partial sums and the coarsest inverse
    nvs = [(8192 // 2 ** k + 1) ** 2 for k in range(13)]     # 8192 .. 2
    L = len(nvs)
    arrays = sum(((5 if k else 3) + (1 if k < L - 1 else 0)) * nv * 8 for k, nv in enumerate(nvs)) + nvs[0] * 8
    assert arrays <= b < arrays + 2 ** 20
    for field, value in (("ndim", 4), ("precision", abi.DMGS_FP32_IN_FP64), ("smoother", abi.DMGS_WJACOBI)):
        ob = abi.default_options(64)
        ob.ndim = 2
        setattr(ob, field, value)
        assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0, field
    for bad in (32768, 20, 1):
        ob = abi.default_options(bad)
        ob.ndim = 2
        assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0, bad
    ob = abi.default_options(2048)
    assert lib.dmgs_workspace_bytes(C.byref(ob)) == 0   # 3D stops at 1024
    ob.ndim = 2
    ob.n[2] = 7                                        # ignored in 2D
    assert lib.dmgs_workspace_bytes(C.byref(ob)) > 0


def test_noalloc_rejections_before_device_work(abi):
    """dmgs_solve_once_noalloc checks its options, pointers and the size of
    the plan against the static scratch array before touching a device (so
    these calls run here, without a GPU)."""
    lib = abi.lib()
    fake = C.c_void_p(0x1000)   # never dereferenced: every call below fails on the host first
    for N, prec, ok_size in ((128, abi.DMGS_FP32_IN_FP64, True), (192, abi.DMGS_FP64, False),
                             (256, abi.DMGS_FP32_IN_FP64, False)):
        o = abi.default_options(N)
        o.precision = prec
        fits = lib.dmgs_workspace_bytes(C.byref(o)) + 64 * 1024 <= abi.DMGS_NOALLOC_SCRATCH_BYTES
        assert fits == ok_size, N
        if not fits:
            st = lib.dmgs_solve_once_noalloc(C.byref(o), fake, fake, fake, fake, None, None)
            assert st == abi.DMGS_ERR_INVALID and "static scratch" in abi.last_error(), N
    o = abi.default_options(32)
    st = lib.dmgs_solve_once_noalloc(C.byref(o), fake, None, fake, fake, None, None)
    assert st == abi.DMGS_ERR_INVALID and "NULL" in abi.last_error()
    o.n[0] = 5
    assert lib.dmgs_solve_once_noalloc(C.byref(o), fake, fake, fake, fake, None, None) == abi.DMGS_ERR_INVALID


def test_status_strings(abi):
    assert abi.status_string(0) == "ok"
    assert abi.status_string(3) == "not converged"


def test_product_path_has_no_oracle_or_fallback():
    """The package never imports the oracle and has no CPU solve path."""
    pkg = os.path.join(ROOT, "paper_2608_00760_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "synth.py", f
                assert "dmgs_ref" not in text, f
