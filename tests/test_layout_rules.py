"""Structural guards (CPU only): the product package never reaches the
oracle, and every GPU test module is marked for the GPU run."""
import ast
import glob
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def test_product_package_does_not_import_the_oracle():
    files = glob.glob(os.path.join(ROOT, "paper_2104_03186_amd", "**", "*.py"), recursive=True)
    assert files
    for f in files:
        for name in _imports(f):
            assert not name.split(".")[0] == "oracle", (f, name)


def test_gpu_test_modules_are_marked():
    for f in glob.glob(os.path.join(ROOT, "tests", "test_gpu_*.py")):
        src = open(f).read()
        assert "pytestmark = pytest.mark.gpu" in src, f
