"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/petar.h, and rejects bad arguments on the host
before any launch (validation-only context, PETAR_NO_DEVICE)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "petar.h")


@pytest.fixture(scope="module")
def capi():
    from paper_2006_16560_amd import _capi
    try:
        return _capi, _capi.load()
    except ImportError as e:
        pytest.skip("libpetar.so not built: %s" % e)


def header_entry_points():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"PETAR_API\s+[\w\s\*]+?\b(petar_\w+)\s*\(", txt)))


def test_exports_every_declared_symbol(capi):
    _capi, lib = capi
    names = header_entry_points()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    declared = {s[0] for s in _capi.SIGNATURES}
    assert set(names) == declared


def test_missing_library_fails_loudly(tmp_path):
    from paper_2006_16560_amd import _capi
    saved = _capi._lib
    _capi._lib = None
    try:
        with pytest.raises(ImportError):
            _capi.load(str(tmp_path / "nope.so"))
    finally:
        _capi._lib = saved


@pytest.fixture()
def ctx(capi):
    _capi, lib = capi
    h = ctypes.c_void_p()
    assert lib.petar_create(ctypes.byref(h), _capi.PETAR_NO_DEVICE, None) == _capi.PETAR_OK
    yield h
    assert lib.petar_destroy(h) == _capi.PETAR_OK


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation-only context


def test_null_ctx(capi):
    _capi, lib = capi
    assert lib.petar_tree_build(None, FAKE, FAKE, 10, 0.5, 8) == _capi.PETAR_E_INVALID
    assert b"ctx" in lib.petar_last_error(None)
    assert lib.petar_create(None, 0, None) == _capi.PETAR_E_INVALID
    assert lib.petar_destroy(None) == _capi.PETAR_E_INVALID


@pytest.mark.parametrize("args,ok", [
    ((FAKE, FAKE, 100, 0.5, 8), True),
    ((None, FAKE, 100, 0.5, 8), False),
    ((FAKE, None, 100, 0.5, 8), False),
    ((FAKE, FAKE, 0, 0.5, 8), False),
    ((FAKE, FAKE, -5, 0.5, 8), False),
    ((FAKE, FAKE, 2 ** 31, 0.5, 8), False),
    ((FAKE, FAKE, 100, -0.1, 8), False),
    ((FAKE, FAKE, 100, float("nan"), 8), False),
    ((FAKE, FAKE, 100, float("inf"), 8), False),
    ((FAKE, FAKE, 100, 0.0, 8), True),
    ((FAKE, FAKE, 100, 0.5, 0), False),
    ((FAKE, FAKE, 100, 0.5, 1), True),
])
def test_tree_build_validation(capi, ctx, args, ok):
    _capi, lib = capi
    st = lib.petar_tree_build(ctx, *args)
    assert st == (_capi.PETAR_E_NODEVICE if ok else _capi.PETAR_E_INVALID)
    if not ok:
        assert lib.petar_last_error(ctx)


def _nb(capi, offsets=FAKE, idx=FAKE, cap=10):
    _capi, _ = capi
    return _capi.petar_nblist(offsets.value if offsets else None, idx.value if idx else None, cap, 0)


@pytest.mark.parametrize("case", ["ok", "ok_nonb", "group0", "rin", "acc", "pot", "nb_off",
                                  "nb_cap", "nb_idx", "nb_cap0"])
def test_force_validation(capi, ctx, case):
    _capi, lib = capi
    args = dict(gs=64, rin=FAKE, rout=FAKE, rs=FAKE, acc=FAKE, pot=FAKE, nb=_nb(capi))
    expect = _capi.PETAR_E_INVALID
    if case == "ok":
        expect = _capi.PETAR_E_NODEVICE
    elif case == "ok_nonb":
        args["nb"] = None
        expect = _capi.PETAR_E_NODEVICE
    elif case == "group0":
        args["gs"] = 0
    elif case == "rin":
        args["rin"] = None
    elif case == "acc":
        args["acc"] = None
    elif case == "pot":
        args["pot"] = None
    elif case == "nb_off":
        args["nb"] = _nb(capi, offsets=None)
    elif case == "nb_cap":
        args["nb"] = _nb(capi, cap=-1)
    elif case == "nb_idx":
        args["nb"] = _nb(capi, idx=None, cap=5)
    elif case == "nb_cap0":
        args["nb"] = _nb(capi, idx=None, cap=0)
        expect = _capi.PETAR_E_NODEVICE
    nbp = ctypes.byref(args["nb"]) if args["nb"] is not None else None
    st = lib.petar_force_long(ctx, args["gs"], args["rin"], args["rout"], args["rs"], args["acc"],
                              args["pot"], nbp)
    assert st == expect, (case, st, lib.petar_last_error(ctx))


@pytest.mark.parametrize("kw,ok", [
    ({}, True),
    ({"G": 0.0}, False),
    ({"G": float("nan")}, False),
    ({"precision": 2}, False),
    ({"precision": 1}, True),
    ({"i_per_lane": 3}, False),
    ({"i_per_lane": 4}, True),
    ({"record_counts": 2}, False),
    ({"workspace_cap": -1}, False),
])
def test_params_validation(capi, ctx, kw, ok):
    _capi, lib = capi
    p = _capi.petar_params()
    assert lib.petar_get_params(ctx, ctypes.byref(p)) == 0
    assert (p.G, p.precision, p.i_per_lane, p.record_counts, p.workspace_cap) == (1.0, 0, 1, 0, 0)
    for k, v in kw.items():
        setattr(p, k, v)
    st = lib.petar_set_params(ctx, ctypes.byref(p))
    assert st == (_capi.PETAR_OK if ok else _capi.PETAR_E_INVALID)


@pytest.mark.parametrize("args,ok", [
    ((FAKE, None, 10, 0.01, 0.1, 1.2, 0.0, FAKE, FAKE, FAKE), True),
    ((FAKE, FAKE, 10, 0.01, 0.1, 1.0, 0.01, FAKE, FAKE, FAKE), True),
    ((None, None, 10, 0.01, 0.1, 1.2, 0.0, FAKE, FAKE, FAKE), False),
    ((FAKE, None, 10, 0.1, 0.1, 1.2, 0.0, FAKE, FAKE, FAKE), False),
    ((FAKE, None, 10, -0.1, 0.1, 1.2, 0.0, FAKE, FAKE, FAKE), False),
    ((FAKE, None, 10, 0.01, 0.1, 0.9, 0.0, FAKE, FAKE, FAKE), False),
    ((FAKE, None, 10, 0.01, 0.1, 1.2, -1.0, FAKE, FAKE, FAKE), False),
    ((FAKE, None, 0, 0.01, 0.1, 1.2, 0.0, FAKE, FAKE, FAKE), False),
    ((FAKE, None, 10, 0.01, 0.1, 1.2, 0.0, None, FAKE, FAKE), False),
])
def test_radii_validation(capi, ctx, args, ok):
    _capi, lib = capi
    st = lib.petar_changeover_radii(ctx, *args)
    assert st == (_capi.PETAR_E_NODEVICE if ok else _capi.PETAR_E_INVALID)


def test_status_strings(capi):
    _capi, lib = capi
    for code in _capi.STATUS_NAMES:
        assert lib.petar_status_string(code)


def test_product_never_touches_oracle():
    """The HIP path and the oracle share no code: no file of the package or
    of the C sources names the oracle."""
    pkg = os.path.join(ROOT, "paper_2006_16560_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "oracle." not in txt, f
                assert "workloads" not in txt, f
    inc = open(HEADER).read()
    assert "oracle" not in inc


def test_autotune_cache_hit_without_device(capi, ctx, tmp_path):
    """A cached entry for (floor(log2 N), theta, precision) is returned without
    any launch; a miss reaches the tree build (no device here)."""
    _capi, lib = capi
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"n_bucket": 20, "theta": 0.5, "precision": 0, "leaf_size": 16, '
                     '"group_size": 128, "i_per_lane": 2, "ms": 3.5}\n'
                     'garbage line\n')
    out = _capi.petar_tuned()
    st = lib.petar_autotune(ctx, FAKE, FAKE, 1 << 20 | 5, 0.5, FAKE, FAKE, FAKE,
                            str(cache).encode(), ctypes.byref(out))
    assert st == _capi.PETAR_OK
    assert (out.leaf_size, out.group_size, out.i_per_lane, out.ms) == (16, 128, 2, 3.5)
    p = _capi.petar_params()
    lib.petar_get_params(ctx, ctypes.byref(p))
    assert p.i_per_lane == 2
    st = lib.petar_autotune(ctx, FAKE, FAKE, 1 << 10, 0.5, FAKE, FAKE, FAKE,
                            str(cache).encode(), ctypes.byref(out))
    assert st == _capi.PETAR_E_NODEVICE
    st = lib.petar_autotune(ctx, None, FAKE, 1 << 10, 0.5, FAKE, FAKE, FAKE, None,
                            ctypes.byref(out))
    assert st == _capi.PETAR_E_INVALID


def test_autotune_lookup_by_n_hint(capi, ctx, tmp_path):
    """petar_autotune_lookup reads a stored choice for (N hint, theta, the
    context's precision) without particles or a device; a miss is
    PETAR_E_STATE, bad arguments PETAR_E_INVALID."""
    _capi, lib = capi
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"n_bucket": 20, "theta": 0.5, "precision": 0, "leaf_size": 16, '
                     '"group_size": 96, "i_per_lane": 2, "ms": 3.5}\n'
                     '{"n_bucket": 20, "theta": 0.5, "precision": 1, "leaf_size": 4, '
                     '"group_size": 32, "i_per_lane": 1, "ms": 9.0}\n')
    out = _capi.petar_tuned()
    path = str(cache).encode()
    assert lib.petar_autotune_lookup(ctx, (1 << 20) + 7, 0.5, path, ctypes.byref(out)) == 0
    assert (out.leaf_size, out.group_size, out.i_per_lane, out.ms) == (16, 96, 2, 3.5)
    p = _capi.petar_params()
    lib.petar_get_params(ctx, ctypes.byref(p))
    p.precision = _capi.PETAR_FP64
    lib.petar_set_params(ctx, ctypes.byref(p))
    assert lib.petar_autotune_lookup(ctx, 1 << 20, 0.5, path, ctypes.byref(out)) == 0
    assert (out.leaf_size, out.group_size, out.i_per_lane) == (4, 32, 1)
    for n_hint, theta in ((1 << 21, 0.5), (1 << 20, 0.3)):
        st = lib.petar_autotune_lookup(ctx, n_hint, theta, path, ctypes.byref(out))
        assert st == _capi.PETAR_E_STATE
    missing = str(tmp_path / "none.jsonl").encode()
    assert lib.petar_autotune_lookup(ctx, 1 << 20, 0.5, missing, ctypes.byref(out)) == \
        _capi.PETAR_E_STATE
    for args in ((0, 0.5, path), (1 << 20, -1.0, path), (1 << 20, 0.5, None)):
        assert lib.petar_autotune_lookup(ctx, *args, ctypes.byref(out)) == _capi.PETAR_E_INVALID


def test_autotune_batch_keys(capi, ctx, tmp_path):
    """Batched choices are keyed by floor(log2 n_sys) besides (floor(log2 N),
    theta, precision): a batch of one system reads the single-system entries
    (written without the field), other system counts only their own; a hit
    of petar_autotune_batch launches nothing, a miss reaches the forest
    build (no device here)."""
    _capi, lib = capi
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"n_bucket": 21, "theta": 0.5, "precision": 0, "leaf_size": 4, '
                     '"group_size": 64, "i_per_lane": 2, "ms": 5.0}\n'
                     '{"n_bucket": 21, "sys_bucket": 7, "theta": 0.5, "precision": 0, '
                     '"leaf_size": 8, "group_size": 96, "i_per_lane": 1, "ms": 12.0}\n')
    path = str(cache).encode()
    out = _capi.petar_tuned()
    n = 3354561  # floor(log2) = 21
    assert lib.petar_autotune_lookup_batch(ctx, n, 128, 0.5, path, ctypes.byref(out)) == 0
    assert (out.leaf_size, out.group_size, out.i_per_lane, out.ms) == (8, 96, 1, 12.0)
    for n_sys in (1, None):
        st = lib.petar_autotune_lookup(ctx, n, 0.5, path, ctypes.byref(out)) if n_sys is None \
            else lib.petar_autotune_lookup_batch(ctx, n, n_sys, 0.5, path, ctypes.byref(out))
        assert st == 0 and (out.leaf_size, out.group_size, out.i_per_lane) == (4, 64, 2)
    assert lib.petar_autotune_lookup_batch(ctx, n, 64, 0.5, path, ctypes.byref(out)) == \
        _capi.PETAR_E_STATE
    assert lib.petar_autotune_lookup_batch(ctx, n, 0, 0.5, path, ctypes.byref(out)) == \
        _capi.PETAR_E_INVALID
    offs = [0] + [n * (k + 1) // 128 for k in range(128)]
    arr = (ctypes.c_int64 * len(offs))(*offs)
    st = lib.petar_autotune_batch(ctx, 128, arr, FAKE, FAKE, 0.5, FAKE, FAKE, FAKE, path,
                                  ctypes.byref(out))
    assert st == _capi.PETAR_OK and (out.leaf_size, out.group_size, out.i_per_lane) == (8, 96, 1)
    p = _capi.petar_params()
    lib.petar_get_params(ctx, ctypes.byref(p))
    assert p.i_per_lane == 1
    # 100 systems: bucket 6, a miss, so the forest build runs (and finds no device)
    offs = [0] + [n * (k + 1) // 100 for k in range(100)]
    arr = (ctypes.c_int64 * len(offs))(*offs)
    st = lib.petar_autotune_batch(ctx, 100, arr, FAKE, FAKE, 0.5, FAKE, FAKE, FAKE, path,
                                  ctypes.byref(out))
    assert st == _capi.PETAR_E_NODEVICE
    bad = (ctypes.c_int64 * 3)(0, 10, 5)  # decreasing offsets: the build rejects them
    assert lib.petar_autotune_batch(ctx, 2, bad, FAKE, FAKE, 0.5, FAKE, FAKE, FAKE, None,
                                    ctypes.byref(out)) == _capi.PETAR_E_INVALID
    for n_sys, a in ((0, arr), (2, None)):
        assert lib.petar_autotune_batch(ctx, n_sys, a, FAKE, FAKE, 0.5, FAKE, FAKE, FAKE, path,
                                        ctypes.byref(out)) == _capi.PETAR_E_INVALID


@pytest.mark.parametrize("offs,ok", [
    ([0, 10, 25], True),
    ([0, 1], True),
    ([1, 10], False),
    ([0, 10, 10], False),
    ([0, 10, 5], False),
])
def test_batch_build_validation(capi, ctx, offs, ok):
    _capi, lib = capi
    arr = (ctypes.c_int64 * len(offs))(*offs)
    st = lib.petar_batch_build(ctx, len(offs) - 1, arr, FAKE, FAKE, 0.5, 8)
    assert st == (_capi.PETAR_E_NODEVICE if ok else _capi.PETAR_E_INVALID)


def test_batch_build_limits(capi, ctx):
    _capi, lib = capi
    offs = list(range(514))
    arr = (ctypes.c_int64 * len(offs))(*offs)
    assert lib.petar_batch_build(ctx, 513, arr, FAKE, FAKE, 0.5, 8) == _capi.PETAR_E_INVALID
    assert lib.petar_batch_build(ctx, 512, arr, FAKE, FAKE, 0.5, 8) == _capi.PETAR_E_NODEVICE
    assert lib.petar_batch_build(ctx, 0, arr, FAKE, FAKE, 0.5, 8) == _capi.PETAR_E_INVALID
    assert lib.petar_batch_build(ctx, 2, None, FAKE, FAKE, 0.5, 8) == _capi.PETAR_E_INVALID


def test_step_graph_validation(capi, ctx):
    _capi, lib = capi
    nb = _nb(capi)
    args = [FAKE, FAKE, 1000, 0.5, 8, 64, FAKE, FAKE, FAKE, FAKE, FAKE]
    assert lib.petar_step_graph(ctx, 0, None, *args, ctypes.byref(nb)) == _capi.PETAR_E_NODEVICE
    assert lib.petar_step_graph(ctx, -1, None, *args, None) == _capi.PETAR_E_INVALID
    bad = list(args)
    bad[4] = 0  # leaf size
    assert lib.petar_step_graph(ctx, 0, None, *bad, None) == _capi.PETAR_E_INVALID
    bad = list(args)
    bad[5] = 0  # group size
    assert lib.petar_step_graph(ctx, 0, None, *bad, None) == _capi.PETAR_E_INVALID
    offs = (ctypes.c_int64 * 3)(0, 5, 5)
    assert lib.petar_step_graph(ctx, 2, offs, *args, None) == _capi.PETAR_E_INVALID


@pytest.mark.parametrize("case", ["ok", "n0", "pos", "vel", "mass", "rnb", "cv0", "cvnan",
                                  "offs", "idx", "out", "out_off", "out_cap", "out_idx"])
def test_nb_filter_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(n=100, pos=FAKE, vel=FAKE, mass=FAKE, rnb=FAKE, cv=1.5, offs=FAKE, idx=FAKE)
    out = _nb(capi)
    if case == "n0":
        a["n"] = 0
    elif case in ("pos", "vel", "mass", "rnb", "offs", "idx"):
        a[case] = None
    elif case == "cv0":
        a["cv"] = 0.0
    elif case == "cvnan":
        a["cv"] = float("nan")
    elif case == "out_off":
        out = _nb(capi, offsets=None)
    elif case == "out_cap":
        out = _nb(capi, cap=-1)
    elif case == "out_idx":
        out = _nb(capi, idx=None)
    outp = None if case == "out" else ctypes.byref(out)
    st = lib.petar_nb_filter(ctx, a["n"], a["pos"], a["vel"], a["mass"], a["rnb"], a["cv"],
                             a["offs"], a["idx"], outp)
    assert st == (_capi.PETAR_E_NODEVICE if case == "ok" else _capi.PETAR_E_INVALID)


@pytest.mark.parametrize("case", ["ok", "n0", "offs", "idx", "label", "cl", "members", "nc"])
def test_clusters_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(n=100, offs=FAKE, idx=FAKE, label=FAKE, cl=FAKE, members=FAKE)
    nc = ctypes.c_int64(0)
    if case == "n0":
        a["n"] = 0
    elif case in a:
        a[case] = None
    ncp = None if case == "nc" else ctypes.byref(nc)
    st = lib.petar_clusters(ctx, a["n"], a["offs"], a["idx"], a["label"], a["cl"], a["members"],
                            ncp)
    assert st == (_capi.PETAR_E_NODEVICE if case == "ok" else _capi.PETAR_E_INVALID)


def _art_set(capi, n_out, null=None):
    _capi, _ = capi
    f = {k: FAKE for k in ("pos_dev", "mass_dev", "r_in_dev", "r_out_dev", "r_search_dev",
                           "src_dev")}
    if null:
        f[null] = None
    return _capi.petar_art_set(n_out=n_out, **f)


@pytest.mark.parametrize("case", ["ok", "ok_no_pairs", "n0", "order", "cd0", "cdnan", "npair_big",
                                  "npair_neg", "pos", "vel", "mass", "rin", "pairs", "frame",
                                  "set", "nout", "set_src", "set_pos"])
def test_artificial_make_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(n=100, pos=FAKE, vel=FAKE, mass=FAKE, rin=FAKE, rout=FAKE, rs=FAKE, npair=10,
             pairs=FAKE, order=3, cd=1.0, frame=FAKE)
    n_out = lambda: a["n"] + a["npair"] * ((4 if a["order"] == 2 else 8) + 2)
    null = None
    if case == "ok_no_pairs":
        a.update(npair=0, pairs=None, frame=None)
    elif case == "n0":
        a["n"] = 0
    elif case == "order":
        a["order"] = 4
    elif case == "cd0":
        a["cd"] = 0.0
    elif case == "cdnan":
        a["cd"] = float("nan")
    elif case == "npair_big":
        a["npair"] = 51
    elif case == "npair_neg":
        a["npair"] = -1
    elif case in ("pos", "vel", "mass", "rin", "pairs", "frame"):
        a[case] = None
    elif case == "set_src":
        null = "src_dev"
    elif case == "set_pos":
        null = "pos_dev"
    s = _art_set(capi, n_out() + (1 if case == "nout" else 0), null)
    st = lib.petar_artificial_make(ctx, a["n"], a["pos"], a["vel"], a["mass"], a["rin"], a["rout"],
                                   a["rs"], a["npair"], a["pairs"], a["order"], a["cd"],
                                   None if case == "set" else ctypes.byref(s), a["frame"], None)
    ok = case in ("ok", "ok_no_pairs")
    assert st == (_capi.PETAR_E_NODEVICE if ok else _capi.PETAR_E_INVALID), lib.petar_last_error(ctx)


@pytest.mark.parametrize("case", ["ok", "ok_tensor_only", "order", "npair", "nout", "acc_set",
                                  "frame", "tensor", "pot_without_acc", "pot_without_pot_set",
                                  "pos", "src", "pairs", "n0"])
def test_tidal_fit_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(order=2, n=100, pos=FAKE, npair=10, pairs=FAKE, frame=FAKE, nout=200, src=FAKE,
             acc_set=FAKE, pot_set=FAKE, tensor=FAKE, acc=FAKE, pot=FAKE)
    if case == "ok_tensor_only":
        a.update(acc=None, pot=None, pos=None, src=None, pairs=None)
    elif case == "order":
        a["order"] = 1
    elif case == "npair":
        a["npair"] = -2
    elif case == "nout":
        a["nout"] = 79  # < 10 * (4 + 4)
    elif case == "pot_without_acc":
        a["acc"] = None
    elif case == "pot_without_pot_set":
        a["pot_set"] = None
    elif case == "n0":
        a["n"] = 0
    elif case in a:
        a[case] = None
    st = lib.petar_tidal_fit(ctx, a["order"], a["n"], a["pos"], a["npair"], a["pairs"], a["frame"],
                             a["nout"], a["src"], a["acc_set"], a["pot_set"], a["tensor"], a["acc"],
                             a["pot"])
    ok = case in ("ok", "ok_tensor_only")
    assert st == (_capi.PETAR_E_NODEVICE if ok else _capi.PETAR_E_INVALID), lib.petar_last_error(ctx)


@pytest.mark.parametrize("case", ["ok", "ok_empty", "order", "npt", "tensor", "frame", "pair_of",
                                  "pos", "acc"])
def test_tidal_eval_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(order=3, npair=5, tensor=FAKE, frame=FAKE, npt=40, pair_of=FAKE, pos=FAKE, acc=FAKE)
    if case == "ok_empty":
        a.update(npt=0, pair_of=None, pos=None, acc=None)
    elif case == "order":
        a["order"] = 0
    elif case == "npt":
        a["npt"] = -1
    elif case in a:
        a[case] = None
    st = lib.petar_tidal_eval(ctx, a["order"], a["npair"], a["tensor"], a["frame"], a["npt"],
                              a["pair_of"], a["pos"], a["acc"], None)
    ok = case in ("ok", "ok_empty")
    assert st == (_capi.PETAR_E_NODEVICE if ok else _capi.PETAR_E_INVALID), lib.petar_last_error(ctx)


@pytest.mark.parametrize("case", ["ok", "n0", "pos", "vel", "mass", "rin", "theta0", "thetanan",
                                  "offs", "idx", "label", "go", "members", "ng", "pairs", "cap",
                                  "np"])
def test_groups_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(n=100, pos=FAKE, vel=FAKE, mass=FAKE, rin=FAKE, theta=0.5, offs=FAKE, idx=FAKE,
             label=FAKE, go=FAKE, members=FAKE, pairs=FAKE, cap=50)
    ng, npair = ctypes.c_int64(0), ctypes.c_int64(0)
    if case == "n0":
        a["n"] = 0
    elif case == "theta0":
        a["theta"] = 0.0
    elif case == "thetanan":
        a["theta"] = float("nan")
    elif case == "cap":
        a["cap"] = 49
    elif case in a:
        a[case] = None
    st = lib.petar_groups(ctx, a["n"], a["pos"], a["vel"], a["mass"], a["rin"], a["theta"],
                          a["offs"], a["idx"], a["label"], a["go"], a["members"],
                          None if case == "ng" else ctypes.byref(ng), a["pairs"], a["cap"],
                          None if case == "np" else ctypes.byref(npair))
    assert st == (_capi.PETAR_E_NODEVICE if case == "ok" else _capi.PETAR_E_INVALID)


@pytest.mark.parametrize("case", ["ok", "n0", "vel", "acc", "dtnan"])
def test_kick_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(n=10, vel=FAKE, acc=FAKE, dt=0.01)
    if case == "n0":
        a["n"] = 0
    elif case == "dtnan":
        a["dt"] = float("inf")
    elif case in a:
        a[case] = None
    st = lib.petar_kick(ctx, a["n"], a["vel"], a["acc"], a["dt"])
    assert st == (_capi.PETAR_E_NODEVICE if case == "ok" else _capi.PETAR_E_INVALID)


@pytest.mark.parametrize("case", ["ok", "vel", "dtinf", "group0", "acc"])
def test_force_long_kick_validation(capi, ctx, case):
    _capi, lib = capi
    a = dict(group=64, vel=FAKE, dt=1e-3, acc=FAKE)
    if case == "vel":
        a["vel"] = None
    elif case == "dtinf":
        a["dt"] = float("inf")
    elif case == "group0":
        a["group"] = 0
    elif case == "acc":
        a["acc"] = None
    st = lib.petar_force_long_kick(ctx, a["group"], FAKE, FAKE, FAKE, a["acc"], FAKE, None,
                                   a["vel"], a["dt"])
    assert st == (_capi.PETAR_E_NODEVICE if case == "ok" else _capi.PETAR_E_INVALID)


def test_set_targets_and_noalloc_validation(capi, ctx):
    """petar_set_targets and petar_clusters_noalloc check their arguments on
    the host: a NULL context, a context without a device, and an N beyond the
    fixed scratch of the no-allocation call (rejected before the device
    check)."""
    _capi, lib = capi
    assert lib.petar_set_targets(None, FAKE) == _capi.PETAR_E_INVALID
    assert lib.petar_set_targets(ctx, FAKE) == _capi.PETAR_E_NODEVICE
    n_cl = ctypes.c_int64(0)
    args = (FAKE, FAKE, FAKE, FAKE, FAKE, ctypes.byref(n_cl))
    assert lib.petar_clusters_noalloc(ctx, (1 << 20) + 1, *args) == _capi.PETAR_E_INVALID
    assert b"fixed scratch" in lib.petar_last_error(ctx)
    assert lib.petar_clusters_noalloc(ctx, 1 << 20, *args) == _capi.PETAR_E_NODEVICE
    assert lib.petar_clusters_noalloc(ctx, 0, *args) == _capi.PETAR_E_INVALID
