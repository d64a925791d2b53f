"""Host-side checks of the test helpers and the benchmark's command line."""
import os
import subprocess
import sys

import numpy as np

import oracle
from helpers import limiter_masks, normwise, rms_rel
from paper_2005_13014_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_limiter_masks_in_fp64_equal_the_oracle_decisions():
    f = inputs.fields(37, 21, 4, 2, seed=3, vadv=False)
    _, _, _, kx, ky = oracle.hdiff(f["u"], 2, f["coeff"], 2, fluxes=True)
    mx, my = limiter_masks(f["u"], 2, "f64")
    assert np.array_equal(kx, mx) and np.array_equal(ky, my)


def test_limiter_masks_fp32_are_float32_decisions():
    # Values exactly representable in float32, so the inputs agree; the
    # decisions may differ from FP64 only where a product sits at rounding level.
    f = inputs.fields(64, 48, 6, 2, seed=4, vadv=False, storage="f32")
    mx, my = limiter_masks(f["u"], 2, "f32")
    _, _, _, kx, ky = oracle.hdiff(f["u"], 2, f["coeff"], 2, fluxes=True)
    flips = int((mx != kx).sum() + (my != ky).sum())
    assert flips <= 3


def test_error_measures():
    ref = np.array([1.0, -2.0, 4.0])
    assert abs(normwise(ref + np.array([0, 0, 4e-6]), ref) - 1e-6) < 1e-15
    assert rms_rel(ref, ref) == 0.0


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_cpu_leg_times_the_oracle_and_checks_kept_outputs():
    """The benchmark's host leg: the oracle timed on a bounded sample, then
    each GPU output it was handed compared with the oracle's result on the
    same inputs (here stand-ins: the exact result and a perturbed copy)."""
    sys.path.insert(0, ROOT)
    import bench
    ni, nj, nk = 20, 9, 6
    f = inputs.fields(ni, nj, nk, 2, seed=bench.SEED + 3, storage="f32")
    ref = oracle.hdiff_vadv(f["u"], 2, f["coeff"], 2, f["wcon"], 2, f["a"], 2, f["b"], 2, f["c"], 2,
                            bench.DT)
    bad = ref.copy()
    bad[1, 2, 3] += 1e-3 * np.abs(ref).max()
    checks = [("exact", "hdiff_vadv", {"f": f, "x": ref}), ("bad", "hdiff_vadv", {"f": f, "x": bad}),
              ("hd", "hdiff", {"f": f, "x": oracle.hdiff(f["u"], 2, f["coeff"], 2)})]
    base, errs = bench.cpu_baseline(ni, nj, nk, checks, budget_s=0.05)
    assert base["kind"] == "oracle" and base["unit"] == "Gpoints/s"
    assert base["cores"] == oracle.threads() >= 1
    assert base["value"] > 0 and base["single_thread_value"] > 0
    assert "%dx%dx%d" % (ni, nj, nk) in base["sample"]
    assert base["host"]["cpu_count"] == os.cpu_count()
    assert errs["exact"] == {"normwise": 0.0, "rms": 0.0} and errs["hd"] == {"normwise": 0.0, "rms": 0.0}
    assert abs(errs["bad"]["normwise"] - 1e-3) < 1e-9 and errs["bad"]["rms"] > 0


def test_bench_timing_statistics():
    sys.path.insert(0, ROOT)
    import bench
    st = bench.stats([4.0, 1.0, 3.0, 2.0, 5.0])
    assert st["median_ms"] == 3.0 and st["q1_ms"] == 2.0 and st["q3_ms"] == 4.0 and st["iqr_ms"] == 2.0
    assert st["mean_ms"] == 3.0 and st["runs"] == 5
    r = bench.record(1.5, [2.0] * 3, points=4e9, nbytes=8e9)
    assert r["Gpoints_s"] == 2000.0 and r["algorithmic_GBs"] == 4000.0 and r["frac_hbm_peak"] == 0.5
    # pooled errors over several outputs
    e = bench.pooled_errors([(np.array([1.0, 2.0]), np.array([1.0, 2.5])), (np.array([4.0]), np.array([4.0]))])
    assert abs(e["normwise"] - 0.5 / 4.0) < 1e-15


def test_product_path_and_oracle_are_independent():
    """The package and the library sources never import, include or link
    the oracle, and the oracle never uses the package's kernels or headers:
    the two share only the seeded input generators."""
    import ast
    import glob
    pkg = os.path.join(ROOT, "paper_2005_13014_amd")
    for path in glob.glob(os.path.join(pkg, "*.py")):
        tree = ast.parse(open(path).read())
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            assert not any(n == "oracle" or n.startswith("oracle.") for n in names), path
    for path in glob.glob(os.path.join(pkg, "csrc", "*")) + glob.glob(os.path.join(ROOT, "include", "*")):
        text = open(path).read()
        assert "oracle" not in text, path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if os.path.isdir(path) or path.endswith((".so", ".o", ".pyc")):
            continue
        text = open(path, errors="replace").read()
        assert "paper_2005_13014_amd.binding" not in text and "libstencil" not in text, path
        assert "csrc" not in text and "stencil.h" not in text, path


def test_missing_library_fails_loudly():
    """Without the built library every entry point raises; there is no
    fallback path (run in a child process so this one's loaded library is
    untouched)."""
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2005_13014_amd import binding as B\n"
        "B.LIB_PATH = '/nonexistent/libstencil.so'\n"
        "try:\n"
        "    B.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not built" in r.stdout
