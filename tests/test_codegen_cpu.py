"""Properties of the generated gfx950 code that the sweep relies on (CPU only;
hipcc cross-compiles).

Regression guard for a memory fault seen with an earlier boundary gather: it
chose face kinds with conditionals over fields of the kernel-argument block, so
the compiler selected between addresses inside that block, and on the
wall-row path the register holding such an address was never written before a
load used it.  Boundary rules are now selects over register copies of the
parameters: the kernels without walls or open faces are straight-line code
(one guard branch); with walls or open faces a kernel adds only its choice of
path per row (plain rows or the general rule), the branch of a plain row's
x-end lanes and the general rule's branches on a cell's own classification
(a solid cell loads nothing, the own state is loaded only next to an open
face); with resolved solid cells, only the branch that skips a solid cell's
loads.  No kernel keeps operands in private memory or writes through the
scalar cache.
"""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2310_14746_amd import build as hbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def asm():
    funcs = {}
    with tempfile.TemporaryDirectory() as tmp:
        for src in ("sweep.hip", "batch.hip", "adjoint.hip"):
            out = os.path.join(tmp, src + ".s")
            cmd = [hbuild.hipcc(), *[f for f in hbuild.HIPCC_FLAGS if f != "-fPIC"],
                   "--cuda-device-only", "-S", os.path.join(hbuild.CSRC, src), "-o", out]
            subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
            text = open(out).read()
            for m in re.finditer(r"^(_Z\w+):.*?\n(.*?)^\.Lfunc_end", text, flags=re.S | re.M):
                funcs[m.group(1)] = m.group(2)
    assert funcs
    return funcs


def _kernels(funcs, prefix):
    return {k: v for k, v in funcs.items() if k.startswith(prefix)}


def _bc(name):
    """Boundary mode of a sweep/reverse-step kernel <L, S, BC, PK> from its mangled name."""
    return int(re.search(r"ELi(\d)ELi\dEEEv", name).group(1))


def _branches(body):
    return len(re.findall(r"^\s+s_(?:c)?branch", body, flags=re.M))


# the guard, the row order's scalar divisions, the choice of path per block,
# the x-end lanes, and in the general rule the skipped loads of a solid cell
# and the own state loaded only next to an open face, each of which the
# compiler may emit as one or two branches
GENERAL_BRANCHES = 12
# the adjoint's seed with walls or open faces: the guard and the general
# rule's two branches
SEED_GENERAL_BRANCHES = 4
# the guard and the skipped loads of a solid cell (one or two branches)
MASKED_BRANCHES = 3


def _allowed(name):
    bc = _bc(name)
    return GENERAL_BRANCHES if bc == 1 else (MASKED_BRANCHES if bc == 2 else 1)


def test_sweep_kernels_are_straight_line(asm):
    sweeps = _kernels(asm, "_ZN4hlbm12sweep_kernel")
    # (2 lattices x 4 storages scalar + 4 storages tensor) x 3 boundary modes
    assert len(sweeps) == 36
    for name, body in sweeps.items():
        assert _branches(body) <= _allowed(name), (name, _branches(body))
    records = _kernels(asm, "_ZN4hlbm19sweep_record_kernel")
    assert len(records) == 24
    for name, body in records.items():
        assert _branches(body) <= _allowed(name), (name, _branches(body))


def test_in_place_kernels_are_straight_line(asm):
    aa = _kernels(asm, "_ZN4hlbm15sweep_aa_kernel")
    # (2 lattices x 4 storages scalar + 4 storages tensor) x 2 step forms x (periodic, walls)
    assert len(aa) == 48
    exports = _kernels(asm, "_ZN4hlbm16aa_export_kernel")
    # 2 lattices x 3 element sizes x (slots of the cell; pulled, periodic; pulled, walls)
    assert len(exports) == 18
    for name, body in {**aa, **exports}.items():
        branches = len(re.findall(r"^\s+s_(?:c)?branch", body, flags=re.M))
        assert branches <= 1, (name, branches)


def test_adjoint_kernels_are_straight_line(asm):
    kern = {**_kernels(asm, "_ZN4hlbm14adjoint_kernel"), **_kernels(asm, "_ZN4hlbm19adjoint_seed_kernel")}
    # reverse step: (2 lattices x 4 storages scalar + 4 storages tensor) x 2 boundary modes;
    # seed: 2 lattices x 4 storages x 2 boundary modes
    assert len(kern) == 24 + 16
    for name, body in kern.items():
        if "adjoint_kernel" in name:
            allowed = GENERAL_BRANCHES if _bc(name) == 1 else 1
        else:
            allowed = SEED_GENERAL_BRANCHES if re.search(r"ELi1EEEv", name) else 1
        assert _branches(body) <= allowed, (name, _branches(body))


def test_no_private_memory_in_sweep_and_moments(asm):
    for name, body in {**_kernels(asm, "_ZN4hlbm12sweep_kernel"),
                       **_kernels(asm, "_ZN4hlbm14moments_kernel"),
                       **_kernels(asm, "_ZN4hlbm14adjoint_kernel"),
                       **_kernels(asm, "_ZN4hlbm17sweep_pair_kernel"),
                       **_kernels(asm, "_ZN4hlbm19sweep_record_kernel"),
                       **_kernels(asm, "_ZN4hlbm17sweep_diag_kernel"),
                       **_kernels(asm, "_ZN4hlbm15sweep_aa_kernel"),
                       **_kernels(asm, "_ZN4hlbm20sweep_aa_diag_kernel"),
                       **_kernels(asm, "_ZN4hlbm19adjoint_seed_kernel"),
                       **_kernels(asm, "_ZN4hlbm23batch_persistent_kernel"),
                       **_kernels(asm, "_ZN4hlbm17batch_step_kernel")}.items():
        assert not re.search(r"^\s+(scratch_|buffer_store|buffer_load)", body, flags=re.M), name


def _arrival_atomic(lines):
    """Index of the grid barrier's arrival atomic: the last atomic add before
    the polling loop (the one with s_sleep)."""
    sleep = next(i for i, l in enumerate(lines) if l.startswith("s_sleep"))
    return max(i for i in range(sleep) if lines[i].startswith("global_atomic_add"))


def test_persistent_barrier_releases_every_wave(asm):
    """Every wave waits for its stores (vmcnt(0)) before the block barrier that
    precedes the arrival count, and the L2 is written back (device-scope
    release) between that barrier and the arrival atomic, so the stores of
    every wave are visible to blocks on other XCDs after the grid barrier."""
    kern = _kernels(asm, "_ZN4hlbm23batch_persistent_kernel")
    assert len(kern) == 8          # four storage forms, each with and without obstacles
    for name, body in kern.items():
        lines = [l.strip() for l in body.splitlines()]
        arrive = _arrival_atomic(lines)
        bar = max(i for i in range(arrive) if lines[i].startswith("s_barrier"))
        before = lines[max(0, bar - 4):bar]
        assert any(l.startswith("s_waitcnt vmcnt(0)") for l in before), name
        between = lines[bar:arrive]
        wb = [i for i, l in enumerate(between) if l.startswith("buffer_wbl2 sc1")]
        assert wb, name
        assert any(l.startswith("s_waitcnt vmcnt(0)") for l in between[wb[0]:]), name


def test_no_scalar_cache_writes(asm):
    for name, body in asm.items():
        assert not re.search(r"^\s+s_(store|atomic|buffer_store|dcache_wb|dcache_discard)", body,
                             flags=re.M), name


_SDEST = re.compile(r"^\s+(?!s_cmp|s_bitcmp|s_cbranch|s_branch|s_waitcnt|s_nop)(?:s_\w+|v_readlane_b32|v_readfirstlane_b32)"
                    r"\s+(?:s\[(\d+):(\d+)\]|s(\d+)\b)")


def _written_in_block(lines, i, regs):
    """Whether every SGPR in `regs` is written between the start of the basic
    block holding line i and line i."""
    left = set(regs)
    for line in reversed(lines[:i]):
        if line.startswith(".LBB") or re.match(r"^\s+s_(?:c)?branch", line):
            break
        m = _SDEST.match(line)
        if m:
            lo, hi = (int(m.group(1)), int(m.group(2))) if m.group(1) else (int(m.group(3)),) * 2
            left -= set(range(lo, hi + 1))
        if not left:
            return True
    return False


def test_no_undefined_sgpr_copied_to_vgpr(asm):
    """No SGPR pair marked implicit-def (undefined on some path) is copied into
    a VGPR pair (the faulting pattern) unless the same basic block writes the
    pair before the copy."""
    for name, body in asm.items():
        undef = set(re.findall(r"implicit-def: \$sgpr(\d+)_sgpr(\d+)", body))
        if not undef:
            continue
        lines = body.splitlines()
        for i, line in enumerate(lines):
            m = re.search(r"v_mov_b64_e32 v\[\d+:\d+\], s\[(\d+):(\d+)\]", line)
            if m and (m.group(1), m.group(2)) in undef:
                assert _written_in_block(lines, i, (int(m.group(1)), int(m.group(2)))), (name, i, line)


def test_block_write_scan_sees_the_faulting_pattern():
    """The scan above on hand-made code: a pair written in the block passes, a
    pair defined only on another path does not."""
    ok = ["\ts_mov_b32 s7, 0x3fac71c7", "\ts_mov_b32 s6, 0x1c71c71c", "\tv_mov_b64_e32 v[68:69], s[6:7]"]
    assert _written_in_block(ok, 2, (6, 7))
    bad = [".LBB0_3:", "\t; implicit-def: $sgpr6_sgpr7", ".LBB0_4:", "\ts_mov_b32 s6, 0",
           "\tv_mov_b64_e32 v[2:3], s[6:7]"]
    assert not _written_in_block(bad, 4, (6, 7))
    wide = ["\ts_load_dwordx4 s[4:7], s[0:1], 0x8", "\tv_mov_b64_e32 v[2:3], s[6:7]"]
    assert _written_in_block(wide, 1, (6, 7))


def test_barrier_polling_keeps_caches(asm):
    """The grid barrier polls with coherent loads and no cache invalidation;
    invalidating the L2 on every poll would evict the data of blocks still
    computing (acquire happens once, after the count is reached)."""
    for name, body in _kernels(asm, "_ZN4hlbm23batch_persistent_kernel").items():
        lines = [l.strip() for l in body.splitlines()]
        add = _arrival_atomic(lines)
        sleep = next(i for i, l in enumerate(lines) if l.startswith("s_sleep"))
        assert add < sleep, name
        window = lines[add:sleep + 40]
        assert not any(l.startswith("buffer_inv") for l in window), name
        # polling loads are device-coherent
        assert any(re.match(r"global_load_dword v\d+, v\d+, s\[\d+:\d+\] sc1", l) for l in window), name
        # and an acquire (invalidate) follows the barrier somewhere in the kernel
        assert any(l.startswith("buffer_inv sc1") for l in lines), name


def test_32bit_offset_helpers_only_index_bounded_rows():
    """ld/st/st_stream form a 32-bit byte offset, which is exact only for rows
    the host bounds below 4 GiB: populations, porosity rows and adjoint
    population rows.  Wider per-cell arrays (FP64 cotangents and gradients,
    the link mask, moments outputs) must use 64-bit indexing, so every call
    of the helpers names one of the bounded arrays."""
    import glob
    bounded = {"src", "dst", "dfield", "f", "lam", "lam_in", "lam_out", "row", "out"}
    seen = set()
    for path in glob.glob(os.path.join(ROOT, "paper_2310_14746_amd", "csrc", "*.hip")) + \
            glob.glob(os.path.join(ROOT, "paper_2310_14746_amd", "csrc", "*.hpp")):
        text = open(path).read()
        for m in re.finditer(r"\b(ld|st|st_stream)\(\s*([A-Za-z_]\w*)", text):
            name = m.group(2)
            if name in ("const", "T"):          # the helpers' own definitions
                continue
            seen.add(name)
            assert name in bounded, (os.path.basename(path), m.group(0))
    assert {"src", "dst", "dfield", "lam"} <= seen
