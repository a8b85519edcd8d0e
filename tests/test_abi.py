"""CPU checks of the C-ABI boundary: the library loads, exports every function declared in
include/qcqp.h, and the ctypes structures match the header's layout (no GPU calls)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qcqp.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qcqp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2605_29291_amd import abi
    L = abi.load()
    names = _declared_functions()
    assert len(names) >= 17, names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(abi.SYMBOLS) == names


def test_defaults_are_the_experiment_settings():
    from paper_2605_29291_amd import abi
    o = abi.default_options()
    # §5: eta = 0.7, c_alpha = 0.4, delta = 0.5 for the yx variants, xi = 0.04, q = 1/2
    assert (o.eta, o.c_alpha, o.delta, o.xi, o.q_restart) == (0.7, 0.4, 0.5, 0.04, 0.5)
    assert o.variant == 0 and o.c_nm == 1 and o.max_iter == 50000 and o.tol == 1e-6


def _c_layout(struct, fields):
    src = "#include <stddef.h>\n#include <stdio.h>\n#include \"qcqp.h\"\nint main(void){\n"
    src += f'printf("%zu\\n", sizeof({struct}));\n'
    for f in fields:
        src += f'printf("%zu\\n", offsetof({struct}, {f}));\n'
    src += "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(cpath, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), cpath, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("cname,pyname", [("qcqp_problem", "Problem"), ("qcqp_options", "Options"),
                                          ("qcqp_info", "Info")])
def test_struct_layouts_match_header(cname, pyname):
    from paper_2605_29291_amd import abi
    S = getattr(abi, pyname)
    fields = [f for f, _ in S._fields_]
    got = _c_layout(cname, fields)
    assert got[0] == C.sizeof(S)
    for f, off in zip(fields, got[1:]):
        assert getattr(S, f).offset == off, f


def test_oracle_and_library_share_nothing():
    """The oracle never loads the HIP library and the library never references the oracle."""
    import oracle
    src = open(os.path.join(ROOT, "oracle", "qcqp_oracle.c")).read()
    assert "qcqp.h" not in src and "hip" not in src.lower().replace("ship", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2605_29291_amd", "csrc")):
        if not f.endswith((".hip", ".h", ".cpp")):
            continue
        text = open(os.path.join(ROOT, "paper_2605_29291_amd", "csrc", f)).read()
        assert "oracle" not in text.lower(), f
    for f in ("__init__.py", "abi.py"):
        text = open(os.path.join(ROOT, "paper_2605_29291_amd", f)).read()
        assert "import oracle" not in text and "from oracle" not in text
    assert oracle.lib() is not None


def test_noalloc_limit_matches_header():
    from paper_2605_29291_amd import abi
    text = open(HEADER).read()
    m = re.search(r"#define\s+QCQP_NOALLOC_MAX_N\s+(\d+)", text)
    assert m and int(m.group(1)) == abi.NOALLOC_MAX_N
