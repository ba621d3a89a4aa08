"""CPU checks of the C ABI: the built library exports every function that
include/pa.h declares, and the argument checks that need no GPU."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from tests.conftest import ROOT


@pytest.fixture(scope="module")
def libpa():
    from paper_2401_07965_amd import build, pa
    if not os.path.exists(pa.LIB_PATH):
        build.build()
    return pa


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pa.h")).read()
    return re.findall(r"^(?:pa_status|void|const char \*)\s*\**\s*(pa_\w+)\s*\(", text, re.M)


def test_header_declares_the_boundary():
    names = set(declared_functions())
    for n in ("pa_init", "pa_sweep", "pa_reweight", "pa_resample", "pa_observables",
              "pa_free_energy", "pa_required_bytes", "pa_export_state", "pa_import_state",
              "pa_overlap", "pa_destroy", "pa_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(libpa):
    so = ctypes.CDLL(libpa.LIB_PATH)
    for n in declared_functions():
        assert hasattr(so, n), n


def test_required_bytes_and_validation_without_gpu(libpa):
    pa = libpa
    small = pa.pa_required_bytes(pa.make_config(2, 8, 1000))
    big = pa.pa_required_bytes(pa.make_config(2, 64, 100000))
    assert 0 < small < big
    # two ping-pong spin buffers of ceil(cap/64) * N words dominate
    cap = 100000 + 8 * 317 + 64
    cap = (cap + 63) // 64 * 64
    assert big >= 2 * (cap // 64) * 4096 * 8
    for bad in (dict(dim=1, L=4, R=10), dict(dim=2, L=3, R=10), dict(dim=2, L=4, R=0),
                dict(dim=2, L=4, R=100, capacity=99), dict(dim=2, L=4, R=10, capacity=1 << 24),
                dict(dim=3, L=26, R=10), dict(dim=2, L=0, R=1)):
        with pytest.raises(pa.PAError) as ei:
            pa.pa_required_bytes(pa.make_config(**bad))
        assert ei.value.status == pa.PA_E_INVAL


def test_spin_packing_roundtrip(libpa):
    pa = libpa
    rng = np.random.default_rng(0)
    for R, N in ((1, 4), (64, 16), (65, 9), (200, 64)):
        s = rng.choice(np.array([-1, 1], np.int8), size=(R, N))
        w = pa.pack_spins(s)
        assert w.shape == ((R + 63) // 64, N)
        assert np.array_equal(pa.unpack_spins(w, R), s)
        # replica r is bit r % 64 of word r // 64; bit 1 means sigma = -1
        r = R - 1
        assert ((int(w[r // 64, 0]) >> (r % 64)) & 1) == (1 if s[r, 0] < 0 else 0)


def test_philox_probe_checks_arguments_without_gpu(libpa):
    L = libpa.lib()
    for n, iters in ((100, 1), (0, 1), (256, 0), ((1 << 24) + 256, 1)):
        assert L.pa_philox_probe(None, n, iters, None) == 1  # PA_E_INVAL, nothing launched


def test_conditional_resampling_calls_check_arguments_without_gpu(libpa):
    L = libpa.lib()
    n = ctypes.c_int64()
    r = ctypes.c_int32()
    # no context: PA_E_INVAL before anything else
    assert L.pa_resample_conditional(None, 2, 0.5, ctypes.byref(n), ctypes.byref(r)) == 1
    assert L.pa_log_weights(None, None, None) == 1


def test_binding_structures_match_the_header(libpa, tmp_path):
    """Sizes and field offsets of every struct the binding mirrors, from the
    header compiled by the C compiler."""
    structs = ("pa_config", "pa_obs", "pa_host_state", "pa_counters", "pa_step_record",
               "pa_combined", "pa_mlp_norm")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pa.h"', 'int main(void) {']
    for s in structs:
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for name, _ in getattr(libpa, s)._fields_:
            lines.append(f'printf("{s}.{name} %zu\\n", offsetof({s}, {name}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                       text=True).stdout.splitlines())
    for s in structs:
        cls = getattr(libpa, s)
        assert int(got[s]) == ctypes.sizeof(cls), s
        for name, _ in cls._fields_:
            assert int(got[f"{s}.{name}"]) == getattr(cls, name).offset, (s, name)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The product path has no fallback: with the HIP library absent, the
    binding raises instead of computing anything another way."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2401_07965_amd import pa\n"
            "pa.LIB_PATH = %r\n"
            "pa._lib = None\n"
            "try:\n"
            "    pa.lib()\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(3)\n") % (ROOT, str(tmp_path / "libpa.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "missing" in r.stdout
