"""The product path never loads the oracle.

The package (binding, build script, training entry) must not import, call or read
anything under oracle/: the oracle is the independent check, not a component.  CPU
part: a syntax-level scan of every package module, and a fresh interpreter that
imports the package and its training entry with `oracle` blocked.  GPU part: the
training entry's own initialisation and a few training iterations on a 16 x 16 toy
problem, again with `oracle` blocked, leave no oracle module loaded."""
import ast
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2011_13926_amd")


def _package_modules():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(dirpath, f)


def test_no_package_module_imports_the_oracle():
    bad = []
    for path in _package_modules():
        tree = ast.parse(open(path).read(), path)
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            elif isinstance(node, ast.Call) and getattr(node.func, "id", "") == "__import__":
                names = [getattr(a, "value", "") for a in node.args[:1]]
            for n in names:
                if str(n).split(".")[0] == "oracle":
                    bad.append((os.path.relpath(path, ROOT), node.lineno, n))
    assert not bad, bad


def test_no_package_source_names_the_oracle_directory():
    """Native sources and build files do not include or read oracle/ either."""
    bad = []
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".hip", ".h", ".cpp", ".py")):
                text = open(os.path.join(dirpath, f)).read()
                if re.search(r"\boracle(/|\.[A-Za-z_])", text):
                    bad.append(os.path.relpath(os.path.join(dirpath, f), ROOT))
    assert not bad, bad


_BLOCKED_IMPORT = r"""
import sys
sys.modules["oracle"] = None          # any `import oracle...` now raises ImportError
sys.path.insert(0, {root!r})
import paper_2011_13926_amd
import paper_2011_13926_amd.train_nn as T
assert not [m for m in sys.modules if m.split(".")[0] == "oracle" and sys.modules[m] is not None]
print("ok")
"""


def test_package_and_training_entry_import_with_the_oracle_blocked():
    if not os.path.exists(os.path.join(PKG, "lib", "libm1.so")):
        pytest.skip("libm1.so not built")
    r = subprocess.run([sys.executable, "-c", _BLOCKED_IMPORT.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr


_BLOCKED_TRAIN = r"""
import sys
sys.modules["oracle"] = None
sys.path.insert(0, {root!r})
import numpy as np
import torch
import paper_2011_13926_amd as P
import paper_2011_13926_amd.train_nn as T
import workloads as W
p = W.voronoi_opacity(n=(16, 16), seed=3, dt=10.0)
pairs = T.generate_pairs(P, torch, p, 1, newton_max=2, partial=(30,))
net, hist = T.train(P, torch, pairs, 20, lr=1e-3, n=16, log_every=0, channels=(16, 16))
w = net.get_params()
assert np.isfinite(w).all() and np.isfinite(hist).all() and len(pairs) >= 2
net.close()
assert not [m for m in sys.modules if m.split(".")[0] == "oracle" and sys.modules[m] is not None]
print("ok", len(pairs), hist[0], hist[-1])
"""


@pytest.mark.gpu
def test_training_runs_with_the_oracle_blocked():
    print("training on a 16x16 toy problem with oracle blocked", flush=True)
    r = subprocess.run([sys.executable, "-c", _BLOCKED_TRAIN.format(root=ROOT)], capture_output=True, text=True,
                       timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0 and "ok" in r.stdout, r.stderr[-4000:]
