"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "c3pt.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(c3pt_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_1711_02384_amd as c
    names = _declared()
    assert "c3pt_spectator_meson" in names and "c3pt_combine" in names
    for n in names:
        assert hasattr(c.lib, n), n
    assert set(names) == set(c.EXPORTED)


def _geom(c, **kw):
    g = c._Geom()
    L = kw.get("L", (4, 4, 4))
    for j in range(3):
        g.L[j] = L[j]
        g.r[j] = 0
    g.T = kw.get("T", 8)
    g.dtype = kw.get("dtype", 0)
    g.proj = kw.get("proj", 0)
    g.stream = None
    return g


def _k(n=1):
    a = np.zeros((n, 3), dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


DUMMY = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("bad", ["L0", "Lbig", "T0", "dtype", "proj", "split_c128", "nmom0", "nmombig",
                                 "noise0", "nullG"])
def test_spectator_rejects_bad_arguments(bad):
    import paper_1711_02384_amd as c
    kw = {}
    n_mom, n_noise, G = 1, 1, DUMMY
    if bad == "L0":
        kw["L"] = (0, 4, 4)
    elif bad == "Lbig":
        kw["L"] = (4, 257, 4)
    elif bad == "T0":
        kw["T"] = 0
    elif bad == "dtype":
        kw["dtype"] = 7
    elif bad == "proj":
        kw["proj"] = 9
    elif bad == "split_c128":
        kw["dtype"], kw["proj"] = 1, 1
    elif bad == "nmom0":
        n_mom = 0
    elif bad == "nmombig":
        n_mom = 257
    elif bad == "noise0":
        n_noise = 0
    elif bad == "nullG":
        G = None
    g = _geom(c, **kw)
    ka, kp = _k(max(n_mom, 1))
    rc = c.lib.c3pt_spectator_meson(ctypes.byref(g), G, DUMMY, n_noise, kp, n_mom, DUMMY)
    assert rc == c.C3PT_EINVAL, (bad, rc)
    assert c.lib.c3pt_last_error().decode()
    rc = c.lib.c3pt_spectator_baryon(ctypes.byref(g), G, DUMMY, DUMMY, n_noise, kp, n_mom, DUMMY)
    assert rc == c.C3PT_EINVAL


def test_insertion_rejects_missing_slices():
    import paper_1711_02384_amd as c
    g = _geom(c, T=4)
    ka, kp = _k(2)
    Gt = (ctypes.c_void_p * 4)(0x1000, 0x1000, None, 0x1000)
    st = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    Ut = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    taus = (ctypes.c_int * 2)(0, 1)
    # local op: slices 0, 1 present -> only a later device error could occur, so
    # test the derivative op, which needs G at tau+1 = 2 (missing)
    rc = c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 1, taus, 2, Ut, 5, kp, 2, DUMMY)
    assert rc == c.C3PT_EINVAL
    assert "needed" in c.lib.c3pt_last_error().decode()
    taus_bad = (ctypes.c_int * 1)(4)
    assert c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 1, taus_bad, 1, None, 1, kp, 2, DUMMY) == c.C3PT_EINVAL
    assert c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 1, taus, 2, None, 5, kp, 2, DUMMY) == c.C3PT_EINVAL
    assert c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 1, taus, 2, None, 3, kp, 2, DUMMY) == c.C3PT_EINVAL
    assert c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 1, taus, 0, None, 1, kp, 2, DUMMY) == c.C3PT_EINVAL


def test_insertion_noalloc_rejects_before_enqueueing():
    """The no-alloc insertion validates and plans on the host: unsupported
    modes and requests whose one timeslice exceeds the fixed scratch are
    rejected before any device call."""
    import paper_1711_02384_amd as c
    assert c.noalloc_scratch_bytes() == 128 << 20
    ka, kp = _k(2)
    Gt = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    st = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    Ut = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    taus = (ctypes.c_int * 2)(0, 1)
    g = _geom(c, T=4)
    g.proj = c.PROJ_NATIVE
    assert c.lib.c3pt_insertion_noalloc(ctypes.byref(g), Gt, st, 1, taus, 2, None, 1, kp, 2, DUMMY) == \
        c.C3PT_EUNSUPPORTED
    g.proj = c.PROJ_FACTORED
    assert c.lib.c3pt_insertion_noalloc(ctypes.byref(g), Gt, st, 1, taus, 2, Ut, 9, kp, 2, DUMMY) == c.C3PT_EINVAL
    assert c.lib.c3pt_insertion_noalloc(ctypes.byref(g), Gt, st, 1, taus, 2, None, 5, kp, 2, DUMMY) == c.C3PT_EINVAL
    Gm = (ctypes.c_void_p * 4)(0x1000, 0x1000, None, 0x1000)
    assert c.lib.c3pt_insertion_noalloc(ctypes.byref(g), Gm, st, 1, taus, 2, Ut, 5, kp, 2, DUMMY) == c.C3PT_EINVAL
    # 256^3 with 64 noise vectors, 5 operators and 123 momenta: one timeslice
    # needs far more partial sums than the fixed array holds
    big = _geom(c, L=(256, 256, 256), T=4)
    big.proj = c.PROJ_FACTORED
    kb = np.ascontiguousarray(np.array(c.momentum_list(9), dtype=np.int32))
    rc = c.lib.c3pt_insertion_noalloc(ctypes.byref(big), Gt, st, 64, taus, 2, Ut, 5,
                                      kb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(kb), DUMMY)
    assert rc == c.C3PT_EINVAL
    msg = c.lib.c3pt_last_error().decode()
    assert "fixed scratch" in msg and str(c.noalloc_scratch_bytes() - 4096) in msg


def test_fused_projection_modes_are_validated():
    """The split-precision fused modes need complex64 inputs and take n_ops 1 or 5."""
    import paper_1711_02384_amd as c
    ka, kp = _k(2)
    Gt = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    st = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    Ut = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    taus = (ctypes.c_int * 2)(0, 1)
    for proj in (c.PROJ_FACTORED_F16, c.PROJ_FACTORED_BF16):
        g = _geom(c, T=4, proj=proj, dtype=1)
        assert c.lib.c3pt_spectator_meson(ctypes.byref(g), DUMMY, DUMMY, 1, kp, 2, DUMMY) == c.C3PT_EINVAL
        g = _geom(c, T=4, proj=proj)
        assert c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 1, taus, 2, Ut, 9, kp, 2, DUMMY) == \
            c.C3PT_EUNSUPPORTED
    g = _geom(c, T=4, proj=6)
    assert c.lib.c3pt_spectator_meson(ctypes.byref(g), DUMMY, DUMMY, 1, kp, 2, DUMMY) == c.C3PT_EINVAL


def test_combine_rejects_bad_arguments():
    import paper_1711_02384_amd as c
    L = c.lib
    pairs = (ctypes.c_int * 4)(0, 0, 3, 0)     # p' = 3 out of range for n_p = 2
    assert L.c3pt_combine(DUMMY, 64, DUMMY, 1, 2, 2, 1, 1, 0, 1, None, pairs, 2, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_combine(DUMMY, 65, DUMMY, 1, 2, 2, 1, 1, 0, 1, None, None, 4, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_combine(DUMMY, 64, DUMMY, 1, 2, 2, 1, 1, 0, 1, None, None, 3, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_combine(DUMMY, 64, DUMMY, 1, 2, 2, 1, 5, 2, 2, None, None, 4, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_combine(DUMMY, 64, DUMMY, 1, 2, 2, 1, 5, 0, 6, None, None, 4, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_combine(None, 64, DUMMY, 1, 2, 2, 1, 1, 0, 1, None, None, 4, DUMMY, None) == c.C3PT_EINVAL


def test_status_strings():
    import paper_1711_02384_amd as c
    for s in (0, -1, -2, -3, -4):
        assert c.lib.c3pt_strerror(s)
    assert c.version() >= 100


def _job(c, **kw):
    j = c._Job()
    j.kind = kw.get("kind", 0)
    L = kw.get("L", (4, 4, 4))
    for d in range(3):
        j.L[d] = L[d]
        j.r[d] = 0
    j.T = kw.get("T", 8)
    j.n_noise = kw.get("n_noise", 1)
    j.G = kw.get("G", DUMMY)
    j.G2 = kw.get("G2", DUMMY)
    j.eta = kw.get("eta", DUMMY)
    j.n_tau = kw.get("n_tau", 0)
    j.n_ops = kw.get("n_ops", 1)
    j.out = kw.get("out", DUMMY)
    return j


@pytest.mark.parametrize("bad", ["empty", "kind", "L0", "T0", "noise0", "out", "G", "baryonG2", "ins_no_tables",
                                 "ins_ops", "nmom0", "nmom129", "proj", "kbig", "comb_index", "comb_kinds",
                                 "comb_ops", "budget"])
def test_batch_rejects_bad_arguments(bad):
    import paper_1711_02384_amd as c
    kw, n_jobs, n_mom, proj, budget = {}, 1, 1, 0, 0
    combs = None
    n_comb = 0
    ka = np.zeros((130, 3), dtype=np.int32)
    if bad == "empty":
        n_jobs = 0
    elif bad == "kind":
        kw["kind"] = 5
    elif bad == "L0":
        kw["L"] = (4, 0, 4)
    elif bad == "T0":
        kw["T"] = 0
    elif bad == "noise0":
        kw["n_noise"] = 0
    elif bad == "out":
        kw["out"] = None
    elif bad == "G":
        kw["G"] = None
    elif bad == "baryonG2":
        kw["kind"], kw["G2"] = 1, None
    elif bad == "ins_no_tables":
        kw["kind"], kw["n_tau"] = 2, 1
    elif bad == "ins_ops":
        kw["kind"], kw["n_tau"], kw["n_ops"] = 2, 1, 3
    elif bad == "nmom0":
        n_mom = 0
    elif bad == "nmom129":
        n_mom = 129
    elif bad == "proj":
        proj = 7
    elif bad == "kbig":
        ka[0, 1] = 40000
    elif bad == "budget":
        budget = 1024          # the job's partial sums need more
    jobs = (c._Job * 2)(_job(c, **kw), _job(c, kind=0))
    if bad.startswith("comb"):
        n_jobs = 2
        combs = (c._CombineJob * 1)()
        cj = combs[0]
        cj.spec_job, cj.ins_job, cj.op_begin, cj.op_end, cj.out = 0, 1, 0, 1, DUMMY
        if bad == "comb_index":
            cj.ins_job = 2
        elif bad == "comb_kinds":
            pass                # job 1 is a spectator, not an insertion
        elif bad == "comb_ops":
            cj.op_end = 0
        n_comb = 1
    handle = ctypes.c_void_p(0x1)
    kp = ka.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    rc = c.lib.c3pt_batch_create(jobs, n_jobs, combs, n_comb, kp, n_mom, proj, budget, ctypes.byref(handle))
    assert rc == c.C3PT_EINVAL, (bad, rc)
    assert not handle.value
    assert c.lib.c3pt_last_error().decode()


def test_batch_null_handles():
    import paper_1711_02384_amd as c
    assert c.lib.c3pt_batch_run(None, None) == c.C3PT_EINVAL
    assert c.lib.c3pt_batch_info(None, None, None, None) == c.C3PT_EINVAL
    assert c.lib.c3pt_batch_destroy(None) == c.C3PT_OK


def test_two_sink_rejects_bad_arguments():
    import paper_1711_02384_amd as c
    g = _geom(c, T=8)
    ka, kp = _k(1)
    full = (ctypes.c_void_p * 8)(*([0x1000] * 8))
    L = c.lib
    args = lambda t_fwd, t_src, t_bwd, n_ops=1, G=full: (ctypes.byref(g), DUMMY, DUMMY, t_fwd, DUMMY, DUMMY, t_bwd,
                                                       t_src, 1, G, full, full, n_ops, kp, 1, None, None, 1,
                                                       DUMMY, DUMMY, DUMMY, DUMMY)
    assert L.c3pt_two_sink_meson(*args(1, 4, 1)) == c.C3PT_EINVAL          # the sinks overlap around T
    assert "overlap" in L.c3pt_last_error().decode()
    assert L.c3pt_two_sink_meson(*args(1, 3, 9)) == c.C3PT_EINVAL          # timeslice outside [0, T)
    assert L.c3pt_two_sink_meson(*args(1, 3, 5, n_ops=21)) == c.C3PT_EINVAL
    holes = (ctypes.c_void_p * 8)(0x1000, 0x1000, None, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    assert L.c3pt_two_sink_meson(*args(1, 3, 5, G=holes)) == c.C3PT_EINVAL
    assert "missing" in L.c3pt_last_error().decode()


def test_insertion_symmetric_and_two_derivative_need_factored_projection_and_slices():
    import paper_1711_02384_amd as c
    L = c.lib
    ka, kp = _k(2)
    taus = (ctypes.c_int * 1)(3)
    full = (ctypes.c_void_p * 8)(*([0x1000] * 8))
    for n_ops in (9, 21):
        g = _geom(c, T=8, proj=0)
        assert L.c3pt_insertion(ctypes.byref(g), full, full, 1, taus, 1, full, n_ops, kp, 2, DUMMY) \
            == c.C3PT_EUNSUPPORTED
    g = _geom(c, T=8, proj=3)
    s_holes = (ctypes.c_void_p * 8)(*[0x1000 if t != 4 else None for t in range(8)])
    assert L.c3pt_insertion(ctypes.byref(g), full, s_holes, 1, taus, 1, full, 9, kp, 2, DUMMY) == c.C3PT_EINVAL
    G_holes = (ctypes.c_void_p * 8)(*[0x1000 if t != 1 else None for t in range(8)])
    assert L.c3pt_insertion(ctypes.byref(g), G_holes, full, 1, taus, 1, full, 21, kp, 2, DUMMY) == c.C3PT_EINVAL
    assert L.c3pt_insertion(ctypes.byref(g), full, full, 1, taus, 1, full, 7, kp, 2, DUMMY) == c.C3PT_EINVAL


def test_gamma_and_smear_reject_bad_arguments():
    import paper_1711_02384_amd as c
    L = c.lib
    m = np.zeros((17, 4, 4), dtype=np.complex128)
    mp = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    # meson: counts outside [1, 16], NULL with a count other than 16, NULL data
    assert L.c3pt_gamma_meson(DUMMY, 1, mp, 17, None, 16, None, 16, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_gamma_meson(DUMMY, 1, None, 4, None, 16, None, 16, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_gamma_meson(None, 1, None, 16, None, 16, None, 16, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_gamma_meson(DUMMY, 0, None, 16, None, 16, None, 16, DUMMY, None) == c.C3PT_EINVAL
    # nucleon: unknown channel, projector counts, NULL projectors with a count other than 2
    assert L.c3pt_gamma_nucleon(DUMMY, 1, 5, None, None, None, 2, None, 16, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_gamma_nucleon(DUMMY, 1, c.PROTON_D, None, None, mp, 17, None, 16, DUMMY, None) == c.C3PT_EINVAL
    assert L.c3pt_gamma_nucleon(DUMMY, 1, c.PROTON_U, None, None, None, 3, None, 16, DUMMY, None) == c.C3PT_EINVAL
    # smearing: negative steps or kappa, missing links, empty field
    g = _geom(c)
    assert L.c3pt_smear(ctypes.byref(g), DUMMY, DUMMY, 4, 12, DUMMY, 0.25, -1) == c.C3PT_EINVAL
    assert L.c3pt_smear(ctypes.byref(g), DUMMY, DUMMY, 4, 12, DUMMY, -0.1, 3) == c.C3PT_EINVAL
    assert L.c3pt_smear(ctypes.byref(g), DUMMY, DUMMY, 4, 12, None, 0.25, 3) == c.C3PT_EINVAL
    assert L.c3pt_smear(ctypes.byref(g), DUMMY, DUMMY, 0, 12, DUMMY, 0.25, 3) == c.C3PT_EINVAL


def test_bench_host_logic():
    """bench.py's host-side helpers: the traffic hash covers the factored
    kernels' planning functions and ignores comments, the recorded traffic
    matches the sources, the
    two-sink pair list has the 185 pairs of 93 momenta."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    api = open(os.path.join(ROOT, "paper_1711_02384_amd", "csrc", "c3pt_api.hip")).read()
    for name in bench.TRAFFIC_FUNCTIONS:
        txt = bench._function_text(api, name)
        assert name + "(" in txt and txt.rstrip().endswith("}")
    h = bench.sources_hash()
    assert len(h) == 16
    for key, (nbytes, hsh) in bench.MEASURED_TRAFFIC.items():
        assert nbytes > 0 and len(hsh) == 16
        assert (bench.measured_traffic(*key) == nbytes) == (hsh == h)
    assert len(bench.pairs_diag_or_zero(93)) == 185
    # comments do not enter the hash; code does
    csrc = os.path.join(ROOT, "paper_1711_02384_amd", "csrc")

    def read_edited(edit):
        def read(name):
            txt = open(os.path.join(csrc, name)).read()
            return edit(txt) if name == "c3pt_fs.h" else txt
        return read
    assert bench.sources_hash(read_edited(lambda t: "// note\n/* block\n comment */\n" + t)) == h
    assert bench.sources_hash(read_edited(lambda t: t + "\nstatic int c3pt_extra_;\n")) != h
    r = bench.roofline_entry("fac_insertion", 1.0e12, 50.0, "fac", traffic=None)
    assert r["bound"] == "alu" and abs(r["achieved"] - 20.0) < 1e-9 and abs(r["frac"] - 20.0 / 78.6) < 1e-4


def test_extent_checks_catch_an_under_sized_buffer():
    """Every call compares, on the host, the bytes its kernels will index with
    the bytes allocated for them before anything is enqueued.  Shrinking the
    allocations in those comparisons (the library's test hook) must make the
    dense, factored, fused and no-alloc paths fail with an extent error, with
    no device call made (the pointers here are never dereferenced).  Halving
    trips the phase tables, which are sized exactly; a factor of a million trips the
    partial sums of every path, sized for the largest momentum group or the
    fixed scratch."""
    import paper_1711_02384_amd as c
    ka, kp = _k(3)
    Gt = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    st = (ctypes.c_void_p * 4)(0x1000, 0x1000, 0x1000, 0x1000)
    taus = (ctypes.c_int * 1)(0)

    def expect(rc, what, case):
        assert rc == c.C3PT_EINVAL, (case, rc)
        msg = c.lib.c3pt_last_error().decode()
        assert "extent check: " + what in msg, (case, msg)

    try:
        c.lib.c3pt_debug_scale_allocations(0.5)
        for dtype in (0, 1):
            g = _geom(c, L=(8, 8, 8), T=4, proj=c.PROJ_NATIVE, dtype=dtype)
            expect(c.lib.c3pt_spectator_meson(ctypes.byref(g), DUMMY, DUMMY, 2, kp, 3, DUMMY), "phase table", dtype)
        g = _geom(c, L=(8, 8, 8), T=4, proj=c.PROJ_FACTORED_F16)
        expect(c.lib.c3pt_spectator_baryon(ctypes.byref(g), DUMMY, DUMMY, DUMMY, 2, kp, 3, DUMMY),
               "split B blocks", "fused baryon")
        c.lib.c3pt_debug_scale_allocations(1e-6)
        for proj, dtype in ((c.PROJ_NATIVE, 0), (c.PROJ_NATIVE, 1), (c.PROJ_FACTORED, 0),
                            (c.PROJ_FACTORED_F16, 0), (c.PROJ_FACTORED_BF16, 0)):
            g = _geom(c, L=(8, 8, 8), T=4, proj=proj, dtype=dtype)
            case = (proj, dtype)
            expect(c.lib.c3pt_spectator_meson(ctypes.byref(g), DUMMY, DUMMY, 2, kp, 3, DUMMY), "partial sums", case)
            expect(c.lib.c3pt_spectator_baryon(ctypes.byref(g), DUMMY, DUMMY, DUMMY, 2, kp, 3, DUMMY),
                   "partial sums", case)
            expect(c.lib.c3pt_insertion(ctypes.byref(g), Gt, st, 2, taus, 1, None, 1, kp, 3, DUMMY),
                   "partial sums", case)
        g = _geom(c, L=(8, 8, 8), T=4, proj=c.PROJ_FACTORED)
        expect(c.lib.c3pt_insertion_noalloc(ctypes.byref(g), Gt, st, 2, taus, 1, None, 1, kp, 3, DUMMY),
               "partial sums", "noalloc")
    finally:
        c.lib.c3pt_debug_scale_allocations(1.0)


def test_shipped_tuning_table_applies_every_entry():
    """Every entry of the tuning table in the package names a variant the
    library has for its (kind, mode, class), and applying the table selects
    it (a typo would otherwise be skipped without a word)."""
    import json

    import paper_1711_02384_amd as c3pt
    with open(c3pt.DEFAULT_TUNING) as f:
        table = json.load(f)
    entries = table["entries"]
    assert c3pt.apply_tuning(table) == len(entries)
    for e in entries:
        assert c3pt.get_variant(e["kind"], e["mode"], e["mt_class"]) == e["variant"], e
