"""The build entry point runs end to end on the CPU: it compiles the HIP
library for gfx950 (here replaced by a stub that records the call, since
the real compile is exercised by every GPU run) and the C oracle, and
imports the binding."""
import os

import __graft_entry__ as entry


def test_build_entry_compiles_the_oracle(monkeypatch):
    from paper_2306_09427_amd import build as pkg_build
    import oracle

    calls = []
    monkeypatch.setattr(pkg_build, "build", lambda *a, **k: calls.append("hip"))
    before = os.path.getmtime(oracle.LIB) if os.path.exists(oracle.LIB) else 0.0
    entry.build()
    assert calls == ["hip"]
    assert os.path.exists(oracle.LIB) and os.path.getmtime(oracle.LIB) >= before
