"""Host logic of the benchmark that decides whether stored counters still
describe the kernel (runs without a GPU)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_hash_ignores_comments_but_not_code(tmp_path):
    b = _bench()
    src = "int f(int x) {\n    // add one\n    return x + 1; /* inline */\n}\n"
    a = tmp_path / "a.hip"
    a.write_text(src)
    c = tmp_path / "c.hip"
    c.write_text("/* header */\nint f(int x) {\n\n    return x + 1;\n}\n// end\n")
    d = tmp_path / "d.hip"
    d.write_text(src.replace("x + 1", "x + 2"))
    assert b.code_sha256(str(a)) == b.code_sha256(str(c))
    assert b.code_sha256(str(a)) != b.code_sha256(str(d))


def test_stored_counters_apply_only_to_their_launch_shape():
    """The committed counter record yields a traffic figure only for the
    precision and lanes it was taken with (and only while the kernel code is
    unchanged, in which case the figure lies between the algorithmic bytes
    and a few times that)."""
    b = _bench()
    t = b.deriv_traffic("adapt", 8)
    if t is not None:
        assert 1.0e9 < t < 3.0e9
    assert b.deriv_traffic("mixed", 8) is None and b.deriv_traffic("adapt", 4) is None
