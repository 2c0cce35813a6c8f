"""Static checks of the repository's boundaries (no GPU).

* The product package (the binding, the autograd operator, the input
  generators, the build script and the HIP sources) never imports or reads
  the oracle: the oracle is test infrastructure.
* The HIP sources and the binding share nothing with the oracle (no file of
  one includes or loads a file of the other).
* bench.py touches the oracle only inside its CPU-baseline worker, and
  __graft_entry__.py only inside smoke().
* No committed file refers to the git-ignored private working folder.
"""
import ast
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORK = "_" + "work"          # the private working folder, spelled so that this file does not name it
PKG = os.path.join(ROOT, "paper_2508_10405_amd")


def _imports(path):
    tree = ast.parse(open(path).read())
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [(a.name, node) for a in node.names]
        elif isinstance(node, ast.ImportFrom):
            out.append((node.module or "", node))
    return tree, out


def test_package_does_not_touch_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        if "_build" in dirpath or "__pycache__" in dirpath:
            continue
        for f in files:
            path = os.path.join(dirpath, f)
            if f.endswith(".py"):
                _, imps = _imports(path)
                assert not [m for m, _ in imps if m.split(".")[0] == "oracle"], path
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(path).read()
                assert not re.search(r"lsrtm_oracle|oracle/", text), path


def _functions_importing_oracle(path):
    tree, imps = _imports(path)
    owners = set()
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    names = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                    if any(n.split(".")[0] == "oracle" for n in names):
                        owners.add(fn.name)
    top = [m for m, node in imps if m.split(".")[0] == "oracle" and node in tree.body]
    return owners, top


def test_bench_and_entry_use_the_oracle_only_where_allowed():
    owners, top = _functions_importing_oracle(os.path.join(ROOT, "bench.py"))
    assert not top and owners == {"cpu_worker"}
    owners, top = _functions_importing_oracle(os.path.join(ROOT, "__graft_entry__.py"))
    assert not top and owners == {"smoke"}


def test_no_committed_file_refers_to_the_working_folder():
    files = subprocess.run(["git", "ls-files"], cwd=ROOT, capture_output=True, text=True).stdout.split()
    if not files:
        return   # not a git checkout
    hits = []
    for f in files:
        if not f.endswith((".py", ".hip", ".h", ".sh", ".toml", ".cfg", ".txt")):
            continue
        text = open(os.path.join(ROOT, f), errors="replace").read()
        if re.search(r"(^|[^A-Za-z0-9])" + WORK + "/", text):
            hits.append(f)
    assert not hits, hits


def test_oracle_does_not_touch_the_gpu_path():
    """The oracle imports only numpy, scipy and the standard library: nothing
    of the package (not even the input generators, which the tests hand it)
    and no compiled library."""
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if not f.endswith(".py"):
            continue
        path = os.path.join(odir, f)
        _, imps = _imports(path)
        roots = {m.split(".")[0] for m, _ in imps}
        assert roots <= {"__future__", "dataclasses", "fractions", "typing", "numpy", "scipy", "math",
                         "functools", "itertools", "collections", ""}, (f, roots)
        text = open(path).read()
        assert "paper_2508_10405_amd" not in text and "liblsrtm" not in text and "ctypes" not in text, f
