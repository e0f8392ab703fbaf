"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/rve_batch.h, mirrors its option struct, and rejects
malformed input on the host before any device call."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2306_09427_amd import binding as rb
from paper_2306_09427_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rve_batch.h")

pytestmark = pytest.mark.skipif(not os.path.exists(rb.LIB_PATH), reason="library not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(rve_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 12
    L = rb.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(rb.EXPORTS)


def test_version_and_defaults():
    assert rb.lib().rve_version() == 1
    o = rb.Opts()
    rb.lib().rve_default_opts(C.byref(o))
    assert o.precision == rb.FP64 and o.alpha == 0.9 and o.n_max == 1_000_000 and o.check_every == 1
    assert o.cg_tol == 1e-6
    assert o.damping == rb.DAMP_VISCOUS and o.energy_check == 0 and o.energy_tol == 0.05
    assert o.floor_tol_rel == 0.0 and o.stall_checks == 16


def test_opts_layout_matches_the_header(tmp_path):
    """The binding's rve_opts mirror has the C struct's size and offsets
    (compiled against include/rve_batch.h with the host compiler)."""
    names = [f[0] for f in rb.Opts._fields_]
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "rve_batch.h"\nint main(void){\n'
                    'printf("%zu\\n", sizeof(rve_opts));\n'
                    + "".join(f'printf("%zu\\n", offsetof(rve_opts, {n}));\n' for n in names) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert out[0] == C.sizeof(rb.Opts)
    assert out[1:] == [getattr(rb.Opts, n).offset for n in names]


def _create(nets, **kw):
    return rb.Batch(nets, **kw)


def _net():
    return synth.pack([synth.voronoi_network(20, [30, 0, 0]), synth.voronoi_network(25, [30, 1, 0])])


@pytest.mark.parametrize("mutate,needle", [
    (lambda b: b.fib.__setitem__((3, 0), 10_000), "out of range"),
    (lambda b: b.fib.__setitem__((4, 1), b.fib[4, 0]), "itself"),
    (lambda b: b.X.__setitem__((0, 1), np.nan), "non-finite"),
    (lambda b: b.is_bnd.__setitem__(slice(None), 0), "no boundary node"),
    (lambda b: b.is_bnd.__setitem__(0, 7), "is_bnd"),
])
def test_malformed_networks_rejected_on_host(mutate, needle):
    b = _net()
    mutate(b)
    with pytest.raises(rb.RVEError) as e:
        _create(b)
    assert e.value.code == rb.EINVAL and needle in str(e.value)


def test_zero_length_fiber_rejected():
    b = _net()
    i, j = b.fib[2]
    b.X[j] = b.X[i]
    with pytest.raises(rb.RVEError) as e:
        _create(b)
    assert e.value.code == rb.EINVAL and "zero length" in str(e.value)


@pytest.mark.parametrize("kw,needle", [
    (dict(alpha=1.5), "alpha"), (dict(alpha=0.0), "alpha"), (dict(c=-1.0), "c must"),
    (dict(check_every=0), "check_every"), (dict(n_max=-1), "n_max"), (dict(precision=7), "precision"),
    (dict(engine=rb.ENGINE_NAIVE, precision=rb.MIXED), "naive"), (dict(threads_per_rve=100), "threads"),
    (dict(EA=0.0), "EA"), (dict(cg_tol=0.0), "cg_tol"), (dict(tol_rel=-1.0), "tolerances"),
    (dict(damping=5), "damping"), (dict(energy_tol=0.0), "energy_tol"),
    (dict(damping=rb.DAMP_ADAPTIVE, precision=rb.MIXED), "FP64 only"),
    (dict(energy_check=True, precision=rb.MIXED), "FP64 only"),
    (dict(damping=rb.DAMP_KINETIC, engine=rb.ENGINE_NAIVE), "naive"),
    (dict(damping=rb.DAMP_ADAPTIVE, engine=rb.ENGINE_NAIVE), "naive"),
    (dict(floor_tol_rel=-1.0), "floor_tol_rel"), (dict(floor_tol_rel=float("inf")), "floor_tol_rel"),
    (dict(floor_tol_rel=1e-5, stall_checks=0), "stall_checks"),
    (dict(floor_tol_rel=1e-5, engine=rb.ENGINE_NAIVE), "stagnation stop"),
    (dict(floor_tol_rel=1e-5, damping=rb.DAMP_KINETIC), "stagnation stop"),
    (dict(floor_tol_rel=1e-5, energy_check=True), "stagnation stop"),
])
def test_bad_options_rejected_on_host(kw, needle):
    with pytest.raises(rb.RVEError) as e:
        _create(_net(), **kw)
    assert e.value.code == rb.EINVAL and needle in str(e.value)


def test_bad_c_per_rve_rejected():
    with pytest.raises(rb.RVEError) as e:
        _create(_net(), c_per_rve=np.array([1.0, -2.0]))
    assert e.value.code == rb.EINVAL and "c_per_rve[1]" in str(e.value)


def test_valid_input_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(rb.RVEError) as e:
        _create(_net())
    assert e.value.code == rb.EDEVICE
