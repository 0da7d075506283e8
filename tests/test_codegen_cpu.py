"""Properties of the generated gfx950 code that the sweep relies on (CPU only;
hipcc cross-compiles).

Regression guard for a memory fault seen with an earlier boundary gather: it
chose face kinds with conditionals over fields of the kernel-argument block, so
the compiler selected between addresses inside that block, and on the
wall-row path the register holding such an address was never written before a
load used it.  The sweep kernels are now straight-line code (one guard branch),
keep no operands in private memory, and never write through the scalar cache.
"""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2310_14746_amd import build as hbuild


@pytest.fixture(scope="module")
def asm():
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "sweep.s")
        cmd = [hbuild.hipcc(), *[f for f in hbuild.HIPCC_FLAGS if f != "-fPIC"],
               "--cuda-device-only", "-S", os.path.join(hbuild.CSRC, "sweep.hip"), "-o", out]
        subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
        text = open(out).read()
    funcs = {}
    for m in re.finditer(r"^(_Z\w+):.*?\n(.*?)^\.Lfunc_end", text, flags=re.S | re.M):
        funcs[m.group(1)] = m.group(2)
    assert funcs
    return funcs


def _kernels(funcs, prefix):
    return {k: v for k, v in funcs.items() if k.startswith(prefix)}


def test_sweep_kernels_are_straight_line(asm):
    sweeps = _kernels(asm, "_ZN4hlbm12sweep_kernel")
    assert len(sweeps) == 16
    for name, body in sweeps.items():
        branches = len(re.findall(r"^\s+s_(?:c)?branch", body, flags=re.M))
        assert branches <= 1, (name, branches)


def test_no_private_memory_in_sweep_and_moments(asm):
    for name, body in {**_kernels(asm, "_ZN4hlbm12sweep_kernel"),
                       **_kernels(asm, "_ZN4hlbm14moments_kernel")}.items():
        assert not re.search(r"^\s+(scratch_|buffer_store|buffer_load)", body, flags=re.M), name


def test_no_scalar_cache_writes(asm):
    for name, body in asm.items():
        assert not re.search(r"^\s+s_(store|atomic|buffer_store|dcache_wb|dcache_discard)", body,
                             flags=re.M), name


def test_no_undefined_sgpr_copied_to_vgpr(asm):
    """No SGPR pair marked implicit-def is copied into a VGPR pair (the faulting pattern)."""
    for name, body in asm.items():
        undef = set(re.findall(r"implicit-def: \$sgpr(\d+)_sgpr(\d+)", body))
        for a, b in undef:
            assert not re.search(r"v_mov_b64_e32 v\[\d+:\d+\], s\[%s:%s\]" % (a, b), body), name
