"""The C-ABI library loads and exports every entry point include/lazyfox.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lazyfox.h")
LIB = os.path.join(ROOT, "paper_2210_03211_amd", "liblazyfox.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lf_create", "lf_destroy", "lf_load_graph", "lf_init_communities",
                     "lf_run_iterations", "lf_get_memberships", "lf_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_entry_point():
    import paper_2210_03211_amd as lf
    names = declared_functions()
    bound = set(dir(lf.Handle)) | set(dir(lf.Batch)) | set(dir(lf.Server))
    # the create calls and lf_last_error are used by the constructors and the error path
    missing = [n for n in names if n not in bound and n not in ("lf_create", "lf_last_error", "lf_batch_create",
                                                                "lf_server_create")]
    assert not missing, missing


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2210_03211_amd._native as nat
    monkeypatch.setattr(nat, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(nat, "_lib", None)
    with pytest.raises(ImportError):
        nat.load_library()


def test_build_flags_disable_contraction_and_packed_fp32():
    from paper_2210_03211_amd import build as b
    assert "-ffp-contract=off" in b.FLAGS
    assert "-packed-fp32-ops" in b.FLAGS
    assert any(f.startswith("--offload-arch=gfx950") for f in b.FLAGS) or b.ARCH != "gfx950"


def test_product_code_never_reaches_the_oracle():
    """The package and its sources neither import nor load anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_2210_03211_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liblfo" not in text and "lfo_" not in text, f


def _imports(path):
    """(module name, enclosing top-level function or None) of every import in a file."""
    import ast
    tree = ast.parse(open(path).read())
    out = []

    def walk(node, fn):
        for ch in ast.iter_child_nodes(node):
            f = ch.name if isinstance(ch, ast.FunctionDef) and fn is None else fn
            if isinstance(ch, ast.Import):
                out.extend((a.name.split(".")[0], f) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom) and ch.module:
                out.append((ch.module.split(".")[0], f))
            walk(ch, f)
    walk(tree, None)
    return out


def test_oracle_users_are_the_allowed_ones():
    """Only the test-side users touch the oracle: the stored expected values are written from
    the oracle and the generator alone (never from the HIP library), the benchmark imports the
    oracle only in its CPU-baseline leg, and the entry file only to build it and in smoke()."""
    golden = _imports(os.path.join(ROOT, "tests", "golden", "make_golden.py"))
    mods = {m for m, _ in golden}
    assert "oracle" in mods and "paper_2210_03211_amd" not in mods and "torch" not in mods
    bench = [(m, f) for m, f in _imports(os.path.join(ROOT, "bench.py")) if m == "oracle"]
    assert bench and all(f == "cpu_baseline" for _, f in bench), bench
    entry = [(m, f) for m, f in _imports(os.path.join(ROOT, "__graft_entry__.py")) if m == "oracle"]
    assert entry and all(f in ("build", "smoke") for _, f in entry), entry


def test_design_notes_cite_existing_tests():
    """Every test the design notes name (as `test_x`, `test_x_*` or file::test_x) and every
    tests/ file they name exists."""
    import glob
    text = open(os.path.join(ROOT, "DESIGN.md")).read()
    src = "".join(open(f).read() for f in glob.glob(os.path.join(ROOT, "tests", "*.py")))
    names = set(re.findall(r"`(test_[a-z0-9_]+)\*?`", text)) | set(re.findall(r"::(test_[a-z0-9_]+)", text))
    files = set(re.findall(r"`tests/([a-z0-9_]+\.py)", text))
    for f in files:
        assert os.path.exists(os.path.join(ROOT, "tests", f)), f
    for n in names:
        if n in {os.path.splitext(f)[0] for f in files}:
            continue
        pat = r"def %s" % re.escape(n) if n.endswith("_") else r"def %s\b" % re.escape(n)
        assert re.search(pat, src), n
