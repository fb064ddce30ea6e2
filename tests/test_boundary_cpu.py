"""Host-side checks of the C ABI that need no GPU: the library loads and exports
every entry point declared in include/racmb.h, and the binding mirrors the
header's structures."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1907_01995_amd import racmb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "racmb.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:rac_status|const char\*)\s+(rac_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_binding_surface():
    assert _declared() == sorted(racmb.EXPORTED)


@pytest.mark.skipif(not racmb.lib_available(), reason="libracmb.so not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(racmb.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not racmb.lib_available(), reason="libracmb.so not built")
def test_status_strings():
    lib = racmb.load()
    assert racmb.status_str(racmb.RAC_ERR_NOT_PD).startswith("block matrix not positive definite")
    assert racmb.status_str(0) == "ok"


def _c_layout(tmp_path):
    """Field offsets and sizes as the C compiler lays out racmb.h's structs."""
    fields = {"rac_problem": [f for f, _ in racmb.Problem_._fields_],
              "rac_opts": [f for f, _ in racmb.Opts_._fields_],
              "rac_result": [f for f, _ in racmb.Result_._fields_]}
    cname = {"lam": "lambda"}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "racmb.h"', "int main(void) {"]
    for st, fs in fields.items():
        src.append('printf("%s size %%zu\\n", sizeof(%s));' % (st, st))
        for f in fs:
            src.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (st, f, st, cname.get(f, f)))
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    out = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        st, f, v = line.split()
        out[(st, f)] = int(v)
    return out


def test_struct_layouts_match_header(tmp_path):
    lay = _c_layout(tmp_path)
    for st, cls in (("rac_problem", racmb.Problem_), ("rac_opts", racmb.Opts_),
                    ("rac_result", racmb.Result_)):
        assert lay[(st, "size")] == C.sizeof(cls), st
        for f, _ in cls._fields_:
            assert lay[(st, f)] == getattr(cls, f).offset, (st, f)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(racmb, "_lib", None)
    monkeypatch.setattr(racmb, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        racmb.load()


@pytest.mark.skipif(not racmb.lib_available(), reason="libracmb.so not built")
@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 200, 2001, 65536])
def test_host_permutation_matches_oracle(n):
    """rac_permutation_host (the library's CPU form of the partition draw) against the
    oracle's, bit for bit; the device form is compared with the oracle in the GPU tests."""
    import numpy as np
    import oracle as O
    rng = np.random.default_rng(n + 1)
    for _ in range(3):
        seed, inst, it = int(rng.integers(0, 2**63)), int(rng.integers(0, 300)), int(rng.integers(0, 5000))
        assert np.array_equal(racmb.permutation_host(seed, inst, it, n), O.permutation(seed, inst, it, n))


@pytest.mark.skipif(not racmb.lib_available(), reason="libracmb.so not built")
def test_host_permutation_rejects_bad_arguments():
    lib = racmb.load()
    out = (C.c_int32 * 4)()
    assert lib.rac_permutation_host(1, 0, 0, 0, out) == racmb.RAC_ERR_ARG
    assert lib.rac_permutation_host(1, 0, -1, 4, out) == racmb.RAC_ERR_ARG
    assert lib.rac_permutation_host(1, 0, 0, 4, None) == racmb.RAC_ERR_ARG
