"""C-ABI checks that need no GPU: the library loads, exports every declared entry point, and
validates plans on the host (no kernel is launched by anything here)."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfc.h")


def _lib():
    from paper_2603_26818_amd import _binding

    if not os.path.exists(_binding.library_path()):
        pytest.skip("libpfc.so not built")
    return _binding, _binding.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("pfc_plan_create", "pfc_fft_r2c", "pfc_fft_c2r", "pfc_step", "pfc_step_backward", "pfc_energy"):
        assert n in names


# entry points that no passage of the paper defines (resource handling, error reporting, launch
# shape): their comment says so instead of citing one
NOT_FROM_THE_PAPER = {"pfc_plan_destroy", "pfc_batch_destroy", "pfc_apfc_destroy", "pfc_status_string",
                      "pfc_last_error", "pfc_batch_check", "pfc_batch_grid"}
CITATION = re.compile(r'Eq\. \(\d|Listing \d|section "')


def test_every_entry_point_cites_its_source():
    """Each declaration block of pfc.h (declarations and the comment above them, up to a blank line)
    carries a "Source:" line that cites the passage of the paper it implements (an equation, a
    listing or a section); the allocation-free step names the callers it is for instead; the
    utilities no passage defines say so."""
    text = open(HEADER).read()
    body = text[text.index("#define PFC_H"):]
    checked = set()
    for block in re.split(r"\n\s*\n", body):
        code = re.sub(r"/\*.*?\*/", "", block, flags=re.S)
        names = set(re.findall(r"\b(pfc_[a-z0-9_]+)\s*\(", code))
        if not names:
            continue
        comment = " ".join(re.findall(r"/\*(.*?)\*/", block, flags=re.S))
        comment = re.sub(r"\s*\n\s*\*?\s*", " ", comment)
        for n in names:
            checked.add(n)
            if n == "pfc_step_noalloc":
                assert "cannot allocate" in comment, n
                continue
            assert "Source:" in comment, f"{n}: no Source line"
            src = comment[comment.index("Source:"):]
            if n in NOT_FROM_THE_PAPER:
                assert "none in the paper" in src, n
            else:
                assert CITATION.search(src), f"{n}: the Source line cites no equation, listing or section"
    assert checked == set(declared_functions())


def test_every_declared_symbol_is_exported():
    _, lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    b, _ = _lib()
    assert set(declared_functions()) <= set(b._SIGS)


def _desc(b, shape=(64, 64), dtype=0, model=0, r=-0.25, dt=0.5, dx=math.pi / 4, flags=0):
    d = b.PlanDesc()
    d.ndim = len(shape)
    for a in range(3):
        d.n[a] = shape[a] if a < len(shape) else 1
        d.dx[a] = dx if a < len(shape) else 1.0
    d.dtype, d.model, d.r, d.dt, d.q1sq, d.R1, d.device, d.flags = dtype, model, r, dt, 2.0, 0.05, 0, flags
    return d


def _create(b, lib, d):
    h = ctypes.c_void_p()
    st = lib.pfc_plan_create(ctypes.byref(h), ctypes.byref(d))
    return st, h


def test_struct_layout_matches_c():
    b, _ = _lib()
    assert ctypes.sizeof(b.PlanDesc) == 104
    assert b.PlanDesc.n.offset == 8 and b.PlanDesc.dx.offset == 32 and b.PlanDesc.r.offset == 64
    assert b.PlanDesc.device.offset == 96 and b.PlanDesc.flags.offset == 100


@pytest.mark.parametrize("shape,dtype", [((64, 64), 0), ((8, 16, 32), 1), ((2048, 2048, 2048), 0), ((4, 4), 1),
                                         ((750, 750, 750), 0), ((30, 20, 12), 1), ((20, 750), 0), ((1400, 1400, 1400), 0)])
def test_plan_create_and_sizes(shape, dtype):
    b, lib = _lib()
    st, h = _create(b, lib, _desc(b, shape, dtype))
    assert st == 0, lib.pfc_last_error()
    npts = math.prod(shape)
    cs = 16 if dtype == 1 else 8
    assert lib.pfc_plan_real_bytes(h) == npts * cs // 2
    # packed: the real field's bytes, with 3D rows longer than one 128-byte line padded to whole lines
    M, CB = shape[-1] // 2, 128 // cs
    Mp = M if (len(shape) == 2 or M <= CB or M % CB == 0) else -(-M // CB) * CB
    assert lib.pfc_plan_state_bytes(h) == npts // shape[-1] * Mp * cs
    assert lib.pfc_plan_half_bytes(h) == npts // shape[-1] * (shape[-1] // 2 + 1) * cs
    ws = lib.pfc_plan_workspace_bytes(h)
    assert ws >= lib.pfc_plan_state_bytes(h) and ws < lib.pfc_plan_state_bytes(h) + (64 << 20)
    assert lib.pfc_plan_destroy(h) == 0


@pytest.mark.parametrize("shape,code", [((64,), 2), ((4, 4, 4, 4), 2), ((48, 64), 2), ((64, 4096), 2), ((2, 64), 2),
                                        ((18, 64), 2), ((6, 22), 2), ((16, 15), 2), ((1050, 8), 2)])
def test_plan_rejects_unsupported_shapes(shape, code):
    b, lib = _lib()
    d = _desc(b, shape[:3])
    d.ndim = len(shape)
    st, h = _create(b, lib, d)
    assert st == code and not h.value
    assert lib.pfc_last_error()


def test_plan_rejects_bad_parameters():
    b, lib = _lib()
    assert _create(b, lib, _desc(b, dt=0.0))[0] == 1
    assert _create(b, lib, _desc(b, dt=float("nan")))[0] == 1
    assert _create(b, lib, _desc(b, dx=0.0))[0] == 1
    assert _create(b, lib, _desc(b, model=7))[0] == 1
    assert _create(b, lib, _desc(b, flags=0x100))[0] == 1
    # r = -1.5: r + L(q) < 0 near q = 1, and dt = 5 makes 1 + dt q (r + L) negative there
    assert _create(b, lib, _desc(b, r=-1.5, dt=5.0))[0] == 1
    assert _create(b, lib, _desc(b, r=-1.5, dt=0.1))[0] == 0


def test_calls_without_workspace_fail_cleanly():
    b, lib = _lib()
    st, h = _create(b, lib, _desc(b))
    assert st == 0
    assert lib.pfc_step(h, None, None, 1, None) == 4  # PFC_ERR_WORKSPACE, before any device call
    assert lib.pfc_plan_set_workspace(h, ctypes.c_void_p(256), 16) == 4  # too small
    assert lib.pfc_plan_set_workspace(h, ctypes.c_void_p(100), 1 << 40) == 3  # misaligned
    lib.pfc_plan_destroy(h)


def test_status_strings():
    _, lib = _lib()
    for code, name in enumerate(["PFC_OK", "PFC_ERR_INVALID_ARG", "PFC_ERR_UNSUPPORTED", "PFC_ERR_ALIGNMENT",
                                 "PFC_ERR_WORKSPACE", "PFC_ERR_HIP", "PFC_ERR_DIVERGED", "PFC_ERR_INTERNAL"]):
        assert lib.pfc_status_string(code).decode() == name


def test_tuning_set_get_validation():
    b, lib = _lib()
    st, h = _create(b, lib, _desc(b, (32, 64, 512), 0))
    assert st == 0
    v = (ctypes.c_int * 5)()
    n = ctypes.c_int()
    assert lib.pfc_plan_get_tuning(h, v, ctypes.byref(n)) == 0 and n.value == 5 and list(v) == [0] * 5
    assert lib.pfc_plan_set_tuning(h, (ctypes.c_int * 5)(1, 1, 1, 1, 1), 5) == 0
    assert lib.pfc_plan_get_tuning(h, v, ctypes.byref(n)) == 0 and list(v) == [1] * 5
    assert lib.pfc_plan_set_tuning(h, (ctypes.c_int * 5)(0, 0, 7, 0, 0), 5) == 1  # no such candidate
    assert lib.pfc_plan_set_tuning(h, (ctypes.c_int * 5)(0, 0, 0, 0, 0), 3) == 1  # 3D has 5 passes
    lib.pfc_plan_destroy(h)
    st, h = _create(b, lib, _desc(b, (8, 4, 8), 0))  # lengths with a single candidate
    assert lib.pfc_plan_set_tuning(h, (ctypes.c_int * 5)(0, 0, 1, 0, 0), 5) == 1
    lib.pfc_plan_destroy(h)


# ---------------------------------------------------------------- complex-amplitude form
def _apfc_desc(b, shape=(64, 64), kvec=None, dtype=0, dB=-0.15, Bx=1.0, t=0.3, v=1.0, dt=0.5, dx=math.pi / 2):
    import pfc_inputs as P

    kvec = P.lattice_vectors("triangular") if kvec is None else kvec
    d = b.ApfcDesc()
    d.ndim = len(shape)
    for a in range(3):
        d.n[a] = shape[a] if a < len(shape) else 1
        d.dx[a] = dx if a < len(shape) else 1.0
    d.dtype = dtype
    d.nfields = len(kvec)
    for j, row in enumerate(kvec):
        for a, c in enumerate(row):
            d.k[j][a] = float(c)
    d.dB, d.Bx, d.t, d.v, d.dt, d.device = dB, Bx, t, v, dt, 0
    return d


def _apfc_create(lib, d):
    h = ctypes.c_void_p()
    return lib.pfc_apfc_create(ctypes.byref(h), ctypes.byref(d)), h


def test_apfc_struct_layout_matches_c():
    b, _ = _lib()
    assert b.ApfcDesc.n.offset == 8 and b.ApfcDesc.dx.offset == 32 and b.ApfcDesc.dtype.offset == 56
    assert b.ApfcDesc.nfields.offset == 60 and b.ApfcDesc.k.offset == 64 and b.ApfcDesc.dB.offset == 832
    assert b.ApfcDesc.dt.offset == 864 and b.ApfcDesc.device.offset == 872 and ctypes.sizeof(b.ApfcDesc) == 880


@pytest.mark.parametrize("lattice,shape,dtype", [("triangular", (64, 64), 0), ("bcc", (256, 256, 256), 0),
                                                 ("fcc2", (30, 20, 12), 1), ("square", (750, 20), 1),
                                                 ("bcc", (2048, 4, 8), 0)])
def test_apfc_create_and_sizes(lattice, shape, dtype):
    import pfc_inputs as P

    b, lib = _lib()
    k = P.lattice_vectors(lattice)
    st, h = _apfc_create(lib, _apfc_desc(b, shape, k, dtype))
    assert st == 0, lib.pfc_last_error()
    n = len(k) * math.prod(shape) * (16 if dtype else 8)
    assert lib.pfc_apfc_field_bytes(h) == n
    assert lib.pfc_apfc_workspace_bytes(h) >= n
    lib.pfc_apfc_destroy(h)


def test_apfc_distinct_products():
    """Distinct products summed one by one (the triples eta_j |eta_i|^2 go into the closed form):
    one triangular shell has the single pair conj(eta_a eta_b) and no other triple; the square
    lattice has neither; bcc has two pairs and two triples of three different amplitudes."""
    import pfc_inputs as P

    b, lib = _lib()
    for lattice, t, expect in [("triangular", 0.3, (1, 0)), ("triangular", 0.0, (0, 0)), ("square", 0.3, (0, 0)),
                               ("bcc", 0.3, (2, 2))]:
        k = P.lattice_vectors(lattice)
        st, h = _apfc_create(lib, _apfc_desc(b, (16,) * k.shape[1], k, t=t))
        assert st == 0
        for j in range(len(P.lattice_vectors(lattice))):
            np_, nt_ = ctypes.c_int(), ctypes.c_int()
            assert lib.pfc_apfc_terms(h, j, ctypes.byref(np_), ctypes.byref(nt_)) == 0
            assert (np_.value, nt_.value) == expect, (lattice, t, j)
        assert lib.pfc_apfc_terms(h, 7, ctypes.byref(np_), ctypes.byref(nt_)) == 1
        lib.pfc_apfc_destroy(h)


def test_apfc_rejects_bad_descriptors():
    import pfc_inputs as P

    b, lib = _lib()
    k3 = P.lattice_vectors("bcc")
    bad = [
        (dict(shape=(18, 64)), 2),             # no schedule for 18
        (dict(shape=(64,)), 1),                # 1D
        (dict(shape=(16, 16, 16)), 1),         # 2D vectors on a 3D grid: k has zero components only if given
        (dict(Bx=-1.0), 1),
        (dict(dt=0.0), 1),
        (dict(dB=-10.0, dt=1.0), 1),           # 1 + dt |k|^2 dB <= 0
        (dict(dx=0.0), 1),
    ]
    for kw, code in bad:
        d = _apfc_desc(b, **kw)
        if kw.get("shape") == (16, 16, 16):
            d.nfields = 1
            for a in range(3):
                d.k[0][a] = 0.0
        st, _ = _apfc_create(lib, d)
        assert st == code, (kw, st, lib.pfc_last_error())
    d = _apfc_desc(b, (8, 8, 8), k3)
    d.nfields = 0
    assert _apfc_create(lib, d)[0] == 1
    d.nfields = 33
    assert _apfc_create(lib, d)[0] == 1


def test_apfc_calls_without_workspace_fail_cleanly():
    b, lib = _lib()
    st, h = _apfc_create(lib, _apfc_desc(b))
    assert st == 0
    buf = ctypes.create_string_buffer(64)
    assert lib.pfc_apfc_step(h, buf, buf, 1, None) == 4  # PFC_ERR_WORKSPACE
    assert lib.pfc_apfc_fft(h, buf, buf, -1, None) == 4
    lib.pfc_apfc_destroy(h)


def test_layout_hint_flags_are_validated():
    """PFC_FLAG_ZBLOCK(s > 0) needs rows of whole lines and a z length that is a power of two >= 256,
    or one whose last-axis schedules step by whole blocks (750 for pairs); unknown flag bits are
    rejected; the state of a paired-plane layout keeps the real field's bytes (plus row padding)."""
    b, lib = _lib()
    ok, h = _create(b, lib, _desc(b, (256, 64, 2048), 1, flags=b.PFC_FLAG_ZBLOCK(3) | b.PFC_FLAG_XROWS_BLOCK))
    assert ok == 0, lib.pfc_last_error()
    assert lib.pfc_plan_state_bytes(h) == 256 * 64 * 1024 * 16
    ok, h = _create(b, lib, _desc(b, (750, 750, 750), 0, flags=b.PFC_FLAG_ZBLOCK(1)))
    assert ok == 0, lib.pfc_last_error()
    assert lib.pfc_plan_state_bytes(h) == 750 * 750 * 384 * 8  # rows of 375 padded to 384
    for shape, zs in (((128, 64, 2048), 1), ((750, 750, 750), 2), ((750, 750, 12), 1), ((16, 32, 64), 1)):
        st, _ = _create(b, lib, _desc(b, shape, 0, flags=b.PFC_FLAG_ZBLOCK(zs)))
        assert st == 1, shape  # PFC_ERR_INVALID_ARG
    st, _ = _create(b, lib, _desc(b, (64, 64), 0, flags=0x100))
    assert st == 1
