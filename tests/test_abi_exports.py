"""The C-ABI library loads on the CPU host and exports every symbol include/pfnks.h declares
(no compute calls: no GPU here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfnks.h")
LIB = os.path.join(ROOT, "paper_2209_08001_amd", "libpfnks.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(pfnks_\w+)\s*\(", text, re.M)))


def test_header_declares_the_step_api():
    names = declared()
    for n in ("pfnks_create_problem", "pfnks_step", "pfnks_energy", "pfnks_mass", "pfnks_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2209_08001_amd import pfnks

    assert sorted(pfnks.EXPORTED) == declared()


def test_workspace_bytes_and_validation_on_host():
    """pfnks_workspace_bytes is pure host arithmetic: sizes and argument errors."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W

    b = pfnks.workspace_bytes((512, 512), W.H, W.DEFAULT_MODEL, W.DEFAULT_SOLVER)
    N = 512 * 512
    assert b >= (31 + 12) * 6 * 8 * N
    # sides: even, >= 4, products of the Fourier radices 2, 3, 5, 7, 11, 13
    for side, tile in ((100, 20), (384, 32), (192, 32), (960, 32), (704, 32), (832, 32), (6, 2), (24, 8)):
        assert pfnks.workspace_bytes((side, side), W.H, W.DEFAULT_MODEL,
                                     dict(W.DEFAULT_SOLVER, tile=(tile, tile, 1), overlap=1)) > 0, side
    for side in (80, 96, 112):
        assert pfnks.workspace_bytes((side,) * 3, W.H, W.DEFAULT_MODEL,
                                     dict(W.DEFAULT_SOLVER, tile=(8, 8, 8), overlap=1)) > 0, side
    for side, tile in ((34, 17), (38, 19), (15, 5), (2, 2), (102, 34)):  # factor 17 or 19, odd, below 4
        with pytest.raises(pfnks.PfnksError):
            pfnks.workspace_bytes((side, side), W.H, W.DEFAULT_MODEL,
                                  dict(W.DEFAULT_SOLVER, tile=(tile, tile, 1), overlap=0))
    with pytest.raises(pfnks.PfnksError):  # a tile that does not divide the side
        pfnks.workspace_bytes((100, 100), W.H, W.DEFAULT_MODEL, W.DEFAULT_SOLVER)
    with pytest.raises(pfnks.PfnksError):
        pfnks.workspace_bytes((64, 64), W.H, W.DEFAULT_MODEL, dict(W.DEFAULT_SOLVER, tile=(48, 48, 1)))


def test_batch_step_rejects_bad_arguments_on_host():
    """pfnks_batch_step validates its arrays before touching any problem."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks

    lib = pfnks.load()
    assert lib.pfnks_batch_step(None, 1, None, 0, None, None) == pfnks.PFNKS_EINVAL
    d = (ctypes.c_double * 1)(0.1)
    hs = (ctypes.c_void_p * 1)(None)
    assert lib.pfnks_batch_step(hs, 1, d, 0, None, None) == pfnks.PFNKS_EINVAL
    assert lib.pfnks_batch_step(hs, -1, d, 0, None, None) == pfnks.PFNKS_EINVAL
    assert lib.pfnks_batch_step(hs, 0, d, 0, None, None) == pfnks.PFNKS_OK


def test_workspace_holds_the_tile_setup():
    """The per-step node blocks of the tile solve (13 values per extended-tile node, every
    tile, in the Krylov element type) are part of the workspace when a Schwarz preconditioner
    is selected, and absent otherwise."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W

    n = (512, 512)
    tiles = (512 // 32) * (512 // 32)
    ext = (32 + 2 * 2) ** 2
    for prec, kb in ((pfnks.FP64, 8), (pfnks.MIXED, 4)):
        s = dict(W.DEFAULT_SOLVER, precision=prec)
        with_tiles = pfnks.workspace_bytes(n, W.H, W.DEFAULT_MODEL, dict(s, pc=pfnks.PC_RAS_SPECTRAL))
        without = pfnks.workspace_bytes(n, W.H, W.DEFAULT_MODEL, dict(s, pc=pfnks.PC_SPECTRAL))
        pack = 13 * tiles * ext * kb
        assert pack <= with_tiles - without <= pack + 4096


def test_create_problem_rejects_on_host():
    """pfnks_create_problem checks its arguments, the workspace size and the log domain of the
    initial state (0 < c < 1, 0 < c eta_i < 1 for i = 1..4 with eta_4 = 4 - eta_1 - eta_2 -
    eta_3) before its first device call.  The workspace address below is 256-aligned and is
    never dereferenced: every case returns before the device is touched."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    import numpy as np

    lib = pfnks.load()
    n = (64, 64)
    N = n[0] * n[1]
    g = pfnks.make_grid(n, W.H)
    m = pfnks.make_model(W.DEFAULT_MODEL)
    s = pfnks.make_solver(W.DEFAULT_SOLVER, 2)
    need = pfnks.workspace_bytes(n, W.H, W.DEFAULT_MODEL, W.DEFAULT_SOLVER)
    fake = ctypes.c_void_p(1 << 30)
    c0, e0 = W.init_fields(n, 3)
    c0 = np.ascontiguousarray(c0, dtype=np.float64).ravel()
    e0 = np.ascontiguousarray(e0, dtype=np.float64).ravel()

    def create(c, e, ws=fake, nbytes=need):
        out = ctypes.c_void_p(12345)
        st = lib.pfnks_create_problem(ctypes.byref(g), ctypes.byref(m), ctypes.byref(s),
                                      None if c is None else pfnks._dp(c), None if e is None else pfnks._dp(e),
                                      ws, ctypes.c_size_t(nbytes), None, ctypes.byref(out))
        return st, out.value

    assert create(None, e0) == (pfnks.PFNKS_EINVAL, 12345)  # out is untouched on a null input
    assert create(c0, e0, ws=ctypes.c_void_p((1 << 30) + 8)) == (pfnks.PFNKS_EINVAL, None)  # misaligned
    assert create(c0, e0, nbytes=need - 1) == (pfnks.PFNKS_ENOSPACE, None)

    def bad_c(v):
        c = c0.copy()
        c[N // 2] = v
        return c

    for v in (0.0, 1.0, -0.1, float("nan")):
        assert create(bad_c(v), e0) == (pfnks.PFNKS_EDOMAIN, None), v
    e = e0.copy()
    e[N + 5] = 0.0  # c eta_2 = 0 at one node
    assert create(c0, e) == (pfnks.PFNKS_EDOMAIN, None)
    e = e0.copy()
    c = c0.copy()
    c[7], e[7], e[N + 7], e[2 * N + 7] = 0.5, 0.4, 0.4, 0.4  # eta_4 = 2.8: c eta_4 = 1.4
    assert create(c, e) == (pfnks.PFNKS_EDOMAIN, None)


def test_residual_static_rejects_on_host():
    """pfnks_residual_static checks its arguments and its scratch limit (2^21 nodes) before the
    first device call (the device addresses below are never dereferenced)."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W

    lib = pfnks.load()
    m = pfnks.make_model(W.DEFAULT_MODEL)
    fake = ctypes.c_void_p(1 << 30)

    def call(n, dt=0.1, ptr=fake):
        g = pfnks.make_grid(n, W.H)
        return lib.pfnks_residual_static(ctypes.byref(g), ctypes.byref(m), 0.17, dt, ptr, ptr, ptr, None, None, None)

    assert call((2048, 2048)) == pfnks.PFNKS_ENOSPACE  # 2^22 nodes
    assert call((256, 128, 128)) == pfnks.PFNKS_ENOSPACE
    assert call((64, 64), dt=0.0) == pfnks.PFNKS_EINVAL
    assert call((64, 64), ptr=None) == pfnks.PFNKS_EINVAL
    assert call((34, 34)) == pfnks.PFNKS_EINVAL


def test_group_rejects_on_host():
    """The lockstep group checks its instance count (1..32), workspace size and every
    instance's initial log domain before its first device call; its workspace is count copies
    of the single-problem layout.  The workspace address below is never dereferenced."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    import numpy as np

    lib = pfnks.load()
    n = (64, 64)
    g = pfnks.make_grid(n, W.H)
    m = pfnks.make_model(W.DEFAULT_MODEL)
    s = pfnks.make_solver(W.DEFAULT_SOLVER, 2)
    one = pfnks.workspace_bytes(n, W.H, W.DEFAULT_MODEL, W.DEFAULT_SOLVER)

    def wsb(count):
        out = ctypes.c_size_t(0)
        st = lib.pfnks_group_workspace_bytes(ctypes.byref(g), ctypes.byref(m), ctypes.byref(s), count,
                                             ctypes.byref(out))
        return st, out.value

    assert wsb(3) == (pfnks.PFNKS_OK, 3 * one)
    assert wsb(32) == (pfnks.PFNKS_OK, 32 * one)
    assert wsb(0)[0] == pfnks.PFNKS_EINVAL
    assert wsb(33)[0] == pfnks.PFNKS_EINVAL
    fields = [W.init_fields(n, s_) for s_ in (1, 2)]
    c0 = np.ascontiguousarray(np.stack([f[0].ravel() for f in fields]))
    e0 = np.ascontiguousarray(np.stack([f[1].ravel() for f in fields]))
    fake = ctypes.c_void_p(1 << 30)

    def create(c, e, count=2, nbytes=2 * one, ws=fake):
        out = ctypes.c_void_p(12345)
        st = lib.pfnks_group_create(ctypes.byref(g), ctypes.byref(m), ctypes.byref(s), count, pfnks._dp(c),
                                    pfnks._dp(e), ws, ctypes.c_size_t(nbytes), None, ctypes.byref(out))
        return st, out.value

    assert create(c0, e0, count=0)[0] == pfnks.PFNKS_EINVAL
    assert create(c0, e0, nbytes=2 * one - 1) == (pfnks.PFNKS_ENOSPACE, None)
    assert create(c0, e0, ws=ctypes.c_void_p((1 << 30) + 8)) == (pfnks.PFNKS_EINVAL, None)
    c = c0.copy()
    c[1, 77] = 1.5  # the second instance leaves the log domain
    assert create(c, e0) == (pfnks.PFNKS_EDOMAIN, None)
    assert lib.pfnks_group_step(None, None, None, None) == pfnks.PFNKS_EINVAL
    assert lib.pfnks_group_set_instance(None, 0, None, None) == pfnks.PFNKS_EINVAL
    assert lib.pfnks_group_get_state(None, 0, None, None) == pfnks.PFNKS_EINVAL
    assert lib.pfnks_group_destroy(None) == pfnks.PFNKS_EINVAL
