"""The C-ABI library on a host without a GPU: it loads, exports every entry
point include/rhg.h declares, and its host-only planning agrees with
the oracle bit for bit.  No device work is launched here."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1501_03545_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_entry_point():
    hdr = open(os.path.join(ROOT, "include", "rhg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = sorted(set(re.findall(r"\b(rhg_[a-z_0-9]+)\s*\(", hdr)) - {"rhg_alloc_fn"})
    assert "rhg_generate" in names and "rhg_emit_edges" in names
    lib = C.CDLL(P.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert P.version().startswith("rhg-mi355x")


CFGS = [(10_000, 6.0, 3.0), (1_000_000, 10.0, 2.7), (100_000_000, 20.0, 2.2), (10_000_000, 16.0, 2.5),
        (1000, 64.0, 2.1), (1_000_000, 4.0, 3.5), (2, 0.5, 2.5), (50, 3.0, 2.05)]


@pytest.mark.parametrize("cfg", CFGS)
def test_plan_matches_oracle_bitwise(cfg):
    n, k, g = cfg
    p = P.rhg_plan(n, k, g, 7)
    a, R = O.solve_R(n, k, g)
    assert p.alpha == a
    assert p.R == R
    assert p.cosh_R == O.cosh(R)
    assert p.n == n and p.seed == 7


def test_plan_matches_oracle_on_batch_parameter_draws():
    rng = np.random.default_rng(4)
    for _ in range(64):
        n = int(round(10 ** (3 + 3 * rng.random())))
        k = 4 + 60 * rng.random()
        g = 2.1 + 1.4 * rng.random()
        p = P.rhg_plan(n, k, g, 0)
        assert (p.alpha, p.R) == O.solve_R(n, k, g)


def test_plan_derived_constants():
    import mpmath as mp
    mp.mp.dps = 50
    p = P.rhg_plan(100_000_000, 20.0, 2.2, 3)
    cR = mp.cosh(mp.mpf(p.R))
    assert abs((mp.mpf(p.cosh_R) + mp.mpf(p.cosh_R_lo)) / cR - 1) < 1e-30
    c = mp.cosh(mp.mpf(p.alpha) * mp.mpf(p.R)) - 1
    assert abs((mp.mpf(p.cosh_aR_m1) + mp.mpf(p.cosh_aR_m1_lo)) / c - 1) < 1e-30


@pytest.mark.parametrize("args,status", [
    ((-1, 6.0, 3.0), P.RHG_EINVAL), ((2**31, 6.0, 3.0), P.RHG_EINVAL), ((1000, 6.0, 2.0), P.RHG_EINVAL),
    ((1000, 6.0, float("nan")), P.RHG_EINVAL), ((1000, 0.0, 3.0), P.RHG_EINVAL),
    ((1000, 999.0, 3.0), P.RHG_EINVAL), ((1000, -3.0, 3.0), P.RHG_EINVAL)])
def test_plan_rejects_invalid_arguments(args, status):
    with pytest.raises(P.RhgError) as ei:
        P.rhg_plan(*args, 1)
    assert ei.value.status == status


def test_plan_reports_unreachable_degree():
    # gamma close to 3.5 at small n: Eq. (22) peaks below the target
    a = O.alpha(3.5)
    peak = max(O.kbar_eq22(200, a, x) for x in np.linspace(0.1, 60, 4000))
    assert peak < 150
    with pytest.raises(P.RhgError) as ei:
        P.rhg_plan(200, 150.0, 3.5, 1)
    assert ei.value.status == P.RHG_ENOROOT


def test_plan_small_n_and_radius_form():
    p0 = P.rhg_plan(0, 5.0, 2.5, 1)
    p1 = P.rhg_plan(1, 5.0, 2.5, 1)
    assert p0.n == 0 and p1.n == 1
    q = P.rhg_plan_radius(1000, 0.8, 5.08, 9)
    assert q.alpha == 0.8 and q.R == 5.08 and math.isnan(q.gamma)
    for bad in [(1000, 0.5, 5.0), (1000, 0.8, 0.0), (1000, 0.8, 90.0), (-5, 0.8, 5.0)]:
        with pytest.raises(P.RhgError):
            P.rhg_plan_radius(*bad, 0)


def test_workspace_size_is_host_only_and_grows_with_n():
    small = P.rhg_index_workspace_bytes(P.rhg_plan(10_000, 6.0, 3.0, 1))
    big = P.rhg_index_workspace_bytes(P.rhg_plan(1_000_000, 10.0, 2.7, 1))
    assert 0 < small < big
    assert big >= 40 * 1_000_000


def test_staging_workspace_follows_the_tuning():
    """Staging (the count pass writes the light rows into slots sized from
    each query's expected degree) is on by default from 2^19 points, and on
    or off on request; the slots add about 4 (2m + 30 n) bytes, sized from
    the plan alone (no device work)."""
    ws = P.rhg_index_workspace_bytes
    small = P.rhg_plan(100_000, 10.0, 2.7, 1)
    assert ws(small) == ws(small, {"stage": -1})
    assert ws(small, {"stage": 1}) > ws(small)
    for n, k, g in ((1 << 20, 20.0, 2.2), (1 << 20, 10.0, 3.0), (4_000_000, 8.0, 2.5)):
        p = P.rhg_plan(n, k, g, 1)
        assert ws(p) == ws(p, {"stage": 1})
        extra = ws(p) - ws(p, {"stage": -1})
        assert 4 * n * (k + 15) < extra < 4 * n * (k + 60), (n, k, g, extra)
        assert ws(p, {"stage_pct": 50}) < ws(p)


def test_row_sort_workspace_and_argument_checks_are_host_only():
    import ctypes as C
    lib = P.load()
    # counters + the list of rows over 8192 entries (at most nnz / 8193 + 1,
    # and at most n) + the map of their 8192-entry tiles
    def bound(n, nnz):
        lcap = min(max(n, 1), nnz // 8193 + 1)
        return 256 + 8 * lcap + 8 * (nnz // 8192 + lcap + 1) + 512
    assert P.rhg_sort_rows_workspace_bytes(0, 0) > 0
    a = P.rhg_sort_rows_workspace_bytes(1_000_000, 10_000_000)
    b = P.rhg_sort_rows_workspace_bytes(1_000_000, 1_000_000_000)
    c = P.rhg_sort_rows_workspace_bytes(10, 10_000_000)  # ten rows of 10^6
    assert 8 * (10_000_000 // 8192) < a < b <= bound(1_000_000, 1_000_000_000)
    assert a <= bound(1_000_000, 10_000_000) and 8 * (10_000_000 // 8192) < c <= bound(10, 10_000_000)
    assert P.rhg_sort_rows_workspace_bytes(-1, 5) == 0
    fake = C.c_void_p(0x1000)
    assert lib.rhg_sort_rows(-1, fake, fake, 5, fake, 1 << 20, None) == P.RHG_EINVAL
    assert lib.rhg_sort_rows(10, fake, fake, -1, fake, 1 << 20, None) == P.RHG_EINVAL
    assert lib.rhg_sort_rows(10, None, fake, 5, fake, 1 << 20, None) == P.RHG_EINVAL
    assert lib.rhg_sort_rows(10, fake, fake, 5, fake, 16, None) == P.RHG_ECAPACITY
    assert lib.rhg_sort_rows(0, None, None, 0, None, 0, None) == P.RHG_OK
    assert lib.rhg_sort_rows(10, None, None, 0, None, 0, None) == P.RHG_OK


def test_long_range_workspace_and_argument_checks_are_host_only():
    import ctypes as C
    lib = P.load()
    a = P.rhg_long_range_workspace_bytes(10**6, 25_000)
    b = P.rhg_long_range_workspace_bytes(10**6, 250_000)
    assert 0 < a < b
    # about 40 B per candidate (2k + 4096 of them, hash table at load <= 1/2)
    # and 48 B per added edge
    J = 2 * 250_000 + 4096
    assert b <= 60 * J + 48 * 250_000 + 16384
    assert P.rhg_long_range_workspace_bytes(-1, 5) == 0 and P.rhg_long_range_workspace_bytes(5, -1) == 0
    fake = C.c_void_p(0x1000)
    big = 1 << 30
    assert lib.rhg_long_range(-1, fake, fake, 0, 1, 1, fake, big, fake, fake, 10, fake, None) == P.RHG_EINVAL
    assert lib.rhg_long_range(10, fake, fake, 0, -1, 1, fake, big, fake, fake, 10, fake, None) == P.RHG_EINVAL
    assert lib.rhg_long_range(10, None, fake, 0, 1, 1, fake, big, fake, fake, 10, fake, None) == P.RHG_EINVAL
    assert lib.rhg_long_range(10, fake, fake, 20, 5, 1, fake, big, fake, fake, 29, fake, None) == P.RHG_ECAPACITY
    assert lib.rhg_long_range(10, fake, fake, 20, 5, 1, fake, 64, fake, fake, 30, fake, None) == P.RHG_ECAPACITY


def _header_structs():
    """Field (name, type, pointer, count) lists of every `typedef struct {...}
    NAME;` in include/rhg.h, comments removed."""
    src = open(os.path.join(ROOT, "include", "rhg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", src, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"^const\s+", "", decl)
            ty, rest = re.match(r"(\w+)\s+(.*)", decl).groups()
            for item in rest.split(","):
                m = re.match(r"(\*?)\s*(\w+)(?:\[(\d+)\])?$", item.strip())
                fields.append((m.group(2), ty, bool(m.group(1)), int(m.group(3) or 1)))
        out[name] = fields
    return out


def test_binding_structs_match_the_header():
    """Every struct the binding mirrors has the header's fields, in order, with
    the same sizes (so the same offsets under natural alignment)."""
    scalar = {"int64_t": C.c_int64, "uint64_t": C.c_uint64, "int32_t": C.c_int32, "double": C.c_double,
              "rhg_status": C.c_int32}
    hs = _header_structs()
    for name in ("rhg_params", "rhg_tuning", "rhg_stats", "rhg_graph_summary", "rhg_csr", "rhg_completion",
                 "rhg_server_stats"):
        cls = getattr(P, name)
        assert [f[0] for f in cls._fields_] == [h[0] for h in hs[name]], name
        for (fname, ftype), (_, hty, ptr, cnt) in zip(cls._fields_, hs[name]):
            if ptr:
                want = C.sizeof(C.c_void_p)
            elif hty in scalar:
                want = C.sizeof(scalar[hty]) * cnt
            else:
                want = C.sizeof(getattr(P, hty)) * cnt
            assert C.sizeof(ftype) == want, (name, fname)


def test_radius_range_is_refused_before_any_device_work():
    """The search's FP32 records and the screen's error bound hold for
    R < 80; a hand-filled rhg_params beyond that is refused by every call
    that takes one (host-side checks, no device work), and the planner
    refuses to produce one."""
    import ctypes as C
    lib = P.load()
    p = P.rhg_plan_radius(1000, 0.75, 79.5, 1)
    E = P.rhg_layout_bands(p)
    assert E[0] == 0.0 and E[-1] == 79.5
    p.R = 85.0  # hand-filled: cosh fields stay as they were
    fake = C.c_void_p(0x1000)
    assert lib.rhg_sample_points(C.byref(p), fake, fake, None) == P.RHG_EINVAL
    assert b"R must be below 80" in lib.rhg_last_error()
    out = C.c_void_p()
    assert lib.rhg_build_index(C.byref(p), fake, fake, None, fake, 1 << 40, 0, C.byref(out), None) == P.RHG_EINVAL
    flag = C.c_void_p(0x2000)
    assert lib.rhg_generate_async(C.byref(p), None, fake, fake, fake, 1 << 40, fake, fake, 10, flag, None) == P.RHG_EINVAL
    b = C.c_int()
    buf = (C.c_double * 65)()
    assert lib.rhg_layout_bands(C.byref(p), None, buf, 65, C.byref(b)) == P.RHG_EINVAL
    with pytest.raises(P.RhgError):
        P.rhg_plan_radius(1000, 0.75, 80.0, 1)
    # a degree so small that Eq. (22) would need R >= 80
    with pytest.raises(P.RhgError) as ei:
        P.rhg_plan(2_000_000_000, 1e-12, 2.5, 1)
    assert ei.value.status in (P.RHG_EINVAL, P.RHG_ENOROOT)


def test_layout_bands_follow_the_tuning():
    p = P.rhg_plan(10**6, 10.0, 2.7, 2)
    E = P.rhg_layout_bands(p, {"inner_radius": 10.0, "band_width": 2.0})
    assert E[:2] == [0.0, 10.0] and E[-1] == p.R
    assert all(0.0 < b - a <= 2.0 + 1e-12 for a, b in zip(E[1:], E[2:]))


def test_temperature_arguments_are_checked_before_any_device_work():
    """The temperature calls refuse T outside (0, 1) and NULL arguments on
    the host; rhg_temp_generate does so before its allocator is called."""
    import ctypes as C
    lib = P.load()
    calls = []

    def _alloc(nbytes, _ctx):
        calls.append(nbytes)
        return None

    cb = P.ALLOC_FN(_alloc)
    out = P.rhg_csr()
    for T in (0.0, -1.0, 1.0, 2.0, float("nan"), float("inf")):
        assert lib.rhg_temp_generate(1000, 6.0, 2.5, T, 1, None, cb, None, 0, C.byref(out), None) == P.RHG_EINVAL
        assert b"temperature" in lib.rhg_last_error()
    assert calls == []
    # a valid T reaches the planner and then the allocator (which fails here)
    assert lib.rhg_temp_generate(1000, 6.0, 2.5, 0.5, 1, None, cb, None, 0, C.byref(out), None) == P.RHG_ENOMEM
    assert lib.rhg_temp_generate(1000, 6.0, 1.5, 0.5, 1, None, cb, None, 0, C.byref(out), None) == P.RHG_EINVAL
    fake = C.c_void_p(0x1000)
    assert lib.rhg_temp_count_edges(None, 0.5, fake, None) == P.RHG_EINVAL
    assert lib.rhg_temp_emit_edges(None, 0.5, fake, fake, 10, 0, None) == P.RHG_EINVAL
