"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/hlbm.h, and validates configurations (no compute calls)."""
import ctypes

import numpy as np
import pytest

from paper_2310_14746_amd import hlbm


@pytest.fixture(scope="module")
def lib():
    return hlbm.load()


def test_exports_every_declared_symbol(lib):
    names = hlbm.declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert lib.hlbm_version() == 3


def test_header_matches_binding_struct():
    # hlbm_config field order in the header equals the ctypes mirror
    import re
    text = open(hlbm.HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} hlbm_config;")]
    fields = re.findall(r"^\s*(?:int|double|void)\s*\*?\s*(\w+)", body, flags=re.M)
    names = []
    for line in body.splitlines():
        m = re.match(r"^\s*(int|double|void)\s*\*?\s*([\w\s,\[\]0-9]+);", line)
        if m:
            for part in m.group(2).split(","):
                names.append(re.sub(r"\[.*\]", "", part).strip())
    assert names == [f[0] for f in hlbm.Config._fields_], (names, fields)


@pytest.mark.parametrize("q", [9, 19])
def test_lattice_tables_match_oracle_set(orc, q):
    c, w = hlbm.lattice_info(q)
    co, wo = orc.lattice(q)
    perm = [int(np.nonzero((co == ci).all(axis=1))[0][0]) for ci in c]
    assert sorted(perm) == list(range(q))
    assert np.allclose(w, wo[perm], rtol=0, atol=1e-17)
    # opposite of i is i+1 for odd i, i-1 for even i > 0
    for i in range(1, q):
        j = i + 1 if i % 2 else i - 1
        assert (c[j] == -c[i]).all()


def _rb(cfg):
    pb, db = ctypes.c_size_t(), ctypes.c_size_t()
    return hlbm.load().hlbm_required_bytes(ctypes.byref(cfg), ctypes.byref(pb), ctypes.byref(db)), pb.value, db.value


def test_required_bytes():
    rc, pb, db = _rb(hlbm.make_config(19, "f32", (256, 256, 256)))
    assert rc == 0 and pb == 19 * 4 * 256 ** 3 and db == 4 * 256 ** 3
    rc, pb, db = _rb(hlbm.make_config(19, "f16s", (64, 32, 16), store_scale=4096.0))
    assert rc == 0 and pb == 19 * 2 * 64 * 32 * 16 and db == 2 * 64 * 32 * 16
    rc, pb, db = _rb(hlbm.make_config(9, "f64", (128, 64, 1), bc_lo=(0, 1, 0), bc_hi=(0, 1, 0)))
    assert rc == 0 and pb == 9 * 8 * 128 * 64 and db == 8 * 128 * 64
    # a tensor control holds six rows
    rc, pb, db = _rb(hlbm.make_config(19, "f32", (32, 16, 8), porosity="tensor"))
    assert rc == 0 and pb == 19 * 4 * 32 * 16 * 8 and db == 6 * 4 * 32 * 16 * 8
    # padded population rows; a scalar control stays one dense row, the six
    # rows of a tensor control take the population pitch
    for st, e in (("f64", 8), ("f32", 4), ("bf16s", 2)):
        rc, pb, db = _rb(hlbm.make_config(19, st, (48, 16, 8), row_pad=8448, store_scale=2.0 ** 10))
        assert rc == 0 and pb == 19 * (e * 48 * 16 * 8 + 8448) and db == e * 48 * 16 * 8
        rc, pb, db = _rb(hlbm.make_config(19, st, (48, 16, 8), row_pad=8448, store_scale=2.0 ** 10,
                                          porosity="tensor"))
        assert rc == 0 and db == 6 * (e * 48 * 16 * 8 + 8448)
    rc, pb, db = _rb(hlbm.make_config(19, "bf16s", (32, 16, 8), porosity="tensor", store_scale=2.0 ** 20))
    assert rc == 0 and db == 6 * 2 * 32 * 16 * 8


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), hlbm.EINVAL),
    (dict(tau=float("nan")), hlbm.EINVAL),
    (dict(shape=(0, 4, 4)), hlbm.EINVAL),
    (dict(lattice=15), hlbm.EINVAL),
    (dict(storage=7), hlbm.EINVAL),
    (dict(bc_lo=(1, 0, 0), bc_hi=(0, 0, 0)), hlbm.EINVAL),
    (dict(bc_lo=(5, 0, 0), bc_hi=(5, 0, 0)), hlbm.EINVAL),
    (dict(storage="f16s", store_scale=3000.0), hlbm.EINVAL),
    (dict(storage="bf16s", store_scale=0.0), hlbm.EINVAL),
    (dict(block_x=96), hlbm.EINVAL),
    (dict(force=(float("inf"), 0, 0)), hlbm.EINVAL),
    (dict(shape=(2048, 2048, 512)), hlbm.EUNSUPPORTED),
    (dict(shape=(8, 70000, 4)), hlbm.EUNSUPPORTED),
    (dict(lattice=9, shape=(8, 8, 2)), hlbm.EINVAL),
    (dict(bc_lo=(1, 0, 0), bc_hi=(1, 0, 0), shape=(2, 8, 8)), hlbm.EINVAL),
    (dict(lattice=9, shape=(8, 8, 1), porosity="tensor"), hlbm.EUNSUPPORTED),
    (dict(pattern="aa", bc_lo=(2, 0, 0), bc_hi=(3, 0, 0)), hlbm.EUNSUPPORTED),
    (dict(pattern="aa", bc_lo=(1, 1, 0), bc_hi=(3, 1, 0)), hlbm.EUNSUPPORTED),
    (dict(pattern="aa", block_x=512), hlbm.EUNSUPPORTED),
    (dict(row_pad=100), hlbm.EINVAL),
    (dict(row_pad=-256), hlbm.EINVAL),
    (dict(row_pad=(1 << 24) + 256), hlbm.EINVAL),
])
def test_config_validation(kw, code):
    args = dict(lattice=19, storage="f32", shape=(16, 16, 16))
    args.update(kw)
    rc, _, _ = _rb(hlbm.make_config(**args))
    assert rc == code
    assert hlbm.load().hlbm_last_error().decode()


def test_unknown_porosity_kind():
    cfg = hlbm.make_config(19, "f32", (16, 16, 16))
    cfg.porosity_kind = 7
    rc, _, _ = _rb(cfg)
    assert rc == hlbm.EINVAL and "porosity_kind" in hlbm.load().hlbm_last_error().decode()


def test_pattern_field():
    # the in-place pattern is accepted for periodic boxes and wall faces and
    # needs the same bytes per population buffer (it keeps one buffer instead
    # of two); open faces are refused
    rc, pb, db = _rb(hlbm.make_config(19, "f32", (64, 32, 16), pattern="aa"))
    assert rc == 0 and pb == 19 * 4 * 64 * 32 * 16
    rc, _, _ = _rb(hlbm.make_config(19, "f32", (64, 32, 16), pattern="aa", bc_lo=(0, 1, 1), bc_hi=(0, 1, 1)))
    assert rc == 0
    rc, _, _ = _rb(hlbm.make_config(9, "f16s", (64, 32, 1), pattern="aa", porosity="scalar"))
    assert rc == 0
    cfg = hlbm.make_config(19, "f32", (16, 16, 16))
    cfg.pattern = 2
    rc, _, _ = _rb(cfg)
    assert rc == hlbm.EINVAL and "pattern" in hlbm.load().hlbm_last_error().decode()


def test_null_arguments(lib):
    assert lib.hlbm_required_bytes(None, None, None) == hlbm.EINVAL
    assert lib.hlbm_create(None, None) == hlbm.EINVAL
    assert lib.hlbm_step(None, 1) == hlbm.EINVAL
    assert lib.hlbm_destroy(None) == hlbm.OK
    assert lib.hlbm_lattice_info(19, None, None) == hlbm.EINVAL


def _batch_rc(items):
    import ctypes as C
    n = len(items)
    arr = (hlbm.Config * n)(*items)
    ctx = C.c_void_p()
    return hlbm.load().hlbm_create_batch(arr, n, C.byref(ctx))


@pytest.mark.parametrize("change,code", [
    (dict(lattice=9, shape=(8, 8, 1)), hlbm.EUNSUPPORTED),
    (dict(storage="f64"), hlbm.EINVAL),          # storage differs from item 0
    (dict(bc_lo=(1, 0, 0), bc_hi=(1, 0, 0)), hlbm.EUNSUPPORTED),
    (dict(shape=(1, 8, 8)), hlbm.EINVAL),
    (dict(shape=(2000, 8, 8)), hlbm.EINVAL),
    (dict(shape=(1000, 1000, 8)), hlbm.EUNSUPPORTED),   # multiply-high quotient bound
    (dict(tau=0.4), hlbm.EINVAL),
    (dict(pattern="aa"), hlbm.EUNSUPPORTED),
    (dict(row_pad=8448), hlbm.EINVAL),        # only items[0] carries the pad
])
def test_batch_validation(change, code):
    base = dict(lattice=19, storage="f32", shape=(32, 32, 32), tau=0.7)
    bad = dict(base)
    bad.update(change)
    assert _batch_rc([hlbm.make_config(**base), hlbm.make_config(**bad)]) == code
    assert hlbm.load().hlbm_last_error().decode()


def test_batch_null_and_count(lib):
    import ctypes as C
    ctx = C.c_void_p()
    assert lib.hlbm_create_batch(None, 1, C.byref(ctx)) == hlbm.EINVAL
    arr = (hlbm.Config * 1)(hlbm.make_config(19, "f32", (16, 16, 16)))
    assert lib.hlbm_create_batch(arr, 0, C.byref(ctx)) == hlbm.EINVAL
    assert lib.hlbm_batch_set_mode(None, 0) == hlbm.EINVAL


def test_batch_quotient_by_multiply_high():
    """The kernels divide by nx and ny with a 32-bit multiply-high by
    ceil(2^32/n); exact whenever l*n < 2^32, which the library checks."""
    for n in (2, 3, 7, 32, 48, 64, 80, 96, 255, 1000, 1024):
        m = ((1 << 32) + n - 1) // n
        lmax = min((1 << 32) // n - 1, 50_000_000)
        ls = np.unique(np.concatenate([np.arange(0, min(lmax, 200_000)),
                                       np.random.default_rng(n).integers(0, lmax, 200_000),
                                       np.array([lmax])])).astype(np.uint64)
        q = (ls * np.uint64(m)) >> np.uint64(32)
        assert np.array_equal(q, ls // np.uint64(n)), n
