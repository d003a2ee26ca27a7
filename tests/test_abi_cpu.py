"""CPU checks of the C ABI boundary: the shared library loads without a GPU and exports
every entry point include/*.h declares; the Python binding mirrors the names; the
product package refuses to run without its HIP library (no CPU fallback)."""
import ctypes as ct
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in ("epidmc.h", "epidmc_denoise.h")]
LIB = os.path.join(ROOT, "paper_2510_24154_amd", "libepidmc.so")


def declared():
    txt = "".join(open(h).read() for h in HEADERS)
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(epidmc_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("epidmc_create", "epidmc_set_phantom_hu", "epidmc_set_epid", "epidmc_set_source_spectrum",
                 "epidmc_set_segments", "epidmc_bind_workspace", "epidmc_run", "epidmc_read_image"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ct.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (epidmc_\w+)", out))
    assert set(declared()) <= exported


def test_binding_mirrors_the_abi():
    import paper_2510_24154_amd as E
    assert set(E.EXPORTS) == set(declared())


def test_no_cpu_fallback_without_library(tmp_path):
    code = ("import paper_2510_24154_amd as E\n"
            "try:\n    E.load_library(%r)\nexcept ImportError as e:\n    print('raised', e)\n" % str(tmp_path / "missing.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "raised" in r.stdout


def test_product_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2510_24154_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "epid_oracle" not in txt, f
