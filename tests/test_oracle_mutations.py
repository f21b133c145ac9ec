"""The oracle's pins are strong enough: each plausible mistake planted in a
temporary copy of the oracle sources (on the CPU) makes some pin fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PIN_FILES = ["tests/test_oracle_path.py", "tests/test_oracle_wmap.py",
             "tests/test_oracle_assign.py", "tests/test_oracle_update.py",
             "tests/test_oracle_soft.py"]

H = "scalp_oracle.c"
S = "scalp_soft_oracle.c"
MUTATIONS = {
    "drop_lambda_term": (H, "float A = c->lambda * dcp + oml * (sc / np);",
                         "float A = oml * (sc / np);"),
    "path_sign": (H, "return d < 0 ? (int)-off : (int)off;", "return d < 0 ? (int)off : (int)-off;"),
    "path_ties_toward_p": (H, "long off = (2 * i * ad + n) / (2 * n);",
                           "long off = (2 * i * ad + n - 1) / (2 * n);"),
    "transposed_centre": (H, "float ey = (float)y - centre[4];", "float ey = (float)y - centre[3];"),
    "spatial_uses_endpoint": (H, "float ex = (float)x - centre[3];", "float ex = (float)x - (float)cx;"),
    "ties_to_last": (H, "if (D < best) { best = D; bestk = k; }", "if (D <= best) { best = D; bestk = k; }"),
    "drop_gamma": (H, "float B = 1.0f + c->gamma * (sw / np);", "float B = 1.0f + (sw / np);"),
    "path_len_excludes_p": (H, "float np = (float)(n + 1);", "float np = (float)(n > 0 ? n : 1);"),
    "wmap_not_squared": (H, "w[i] = (float)(1.0 - exp(-(c * c) / s2));", "w[i] = (float)(1.0 - exp(-c / s2));"),
    "missing_neighbour": (H, "for (int dj = -1; dj <= 1; dj++) {", "for (int dj = -1; dj <= 0; dj++) {"),
    "update_x_from_row": (H, "sx[k] += p % W;", "sx[k] += p / W;"),
    "projection_ties": (H, "if (d < best) { best = d; bestp = p; }", "if (d <= best) { best = d; bestp = p; }"),
    "cell_rounding": (H, "static int cell_col(int x, int W, int nx) { return (int)(((long)x * nx) / W); }",
                      "static int cell_col(int x, int W, int nx) { return (int)(((long)x * nx + W / 2) / W); }"),
    "window_off_by_one": (H, "if (abs(x - wx[k]) > R) continue;",
                          "if (abs(x - wx[k]) >= R) continue;"),
    "window_rows_off_by_one": (H, "if (abs(y - wy[k]) <= R) rowk[nk++] = k;",
                               "if (abs(y - wy[k]) < R) rowk[nk++] = k;"),
    "window_ties_to_last": (H, "if (D < best) {       /* ascending k", "if (D <= best) {       /* ascending k"),
    "soft_bwd_drop_lambda": (S, "double cfp = R(r32, R(r32, g * Bw) * lambda);",
                             "double cfp = 0.0 * R(r32, R(r32, g * Bw) * lambda);"),
    "soft_bwd_drop_gamma": (S, "double cwq = R(r32, R(r32, R(r32, g * A) * c.gamma) / np);",
                            "double cwq = R(r32, R(r32, g * A) / np);"),
    "soft_bwd_softmax_sign": (S, "double g = R(r32, -R(r32, R(r32, 1.0 / T) * Q[9 * p + j]) *",
                              "double g = R(r32, R(r32, R(r32, 1.0 / T) * Q[9 * p + j]) *"),
}


# Pin files that are expected to catch each family of mistakes (all files
# are run for a mutation not listed here).
WHERE = {
    "soft_bwd_drop_lambda": ["tests/test_oracle_soft.py"],
    "soft_bwd_drop_gamma": ["tests/test_oracle_soft.py"],
    "soft_bwd_softmax_sign": ["tests/test_oracle_soft.py"],
    "update_x_from_row": ["tests/test_oracle_update.py"],
    "projection_ties": ["tests/test_oracle_update.py"],
    "wmap_not_squared": ["tests/test_oracle_wmap.py"],
    "window_off_by_one": ["tests/test_oracle_window.py"],
    "window_rows_off_by_one": ["tests/test_oracle_window.py"],
    "window_ties_to_last": ["tests/test_oracle_window.py"],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    fname, old, new = MUTATIONS[name]
    work = tmp_path / "oracle"
    shutil.copytree(ORACLE, work, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = (work / fname).read_text()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    (work / fname).write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle.oracle import CFLAGS, _SOURCES
    lib = work / "liboracle_mut.so"
    subprocess.run(["gcc", *CFLAGS, "-o", str(lib), *[str(work / s) for s in _SOURCES], "-lm"],
                   check=True)
    env = dict(os.environ, SCALP_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *WHERE.get(name, PIN_FILES)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, (
        f"planted mistake '{name}' survived the pins:\n{r.stdout[-2000:]}")


# Mistakes planted in the numpy parts of the oracle (quality metrics and
# per-pixel maps), with the pin file expected to catch each.
PM = "metrics.py"
PP = "maps.py"
PY_MUTATIONS = {
    "br_radius_inclusive": (PM, "if dx * dx + dy * dy >= eps * eps:", "if dx * dx + dy * dy > eps * eps:"),
    "br_square_window": (PM, "if dx * dx + dy * dy >= eps * eps:", "if False:"),
    "asa_sum_not_max": (PM, "t.max(axis=1).sum()", "t.sum(axis=1).max()"),
    "ue_counts_every_region": (PM, "((size - t) * (t > 0)).sum()", "(size - t).sum()"),
    "co_no_border_edges": (PM, "edges += np.bincount(L[0, :], minlength=K) + np.bincount(L[-1, :], minlength=K)",
                           "pass"),
    "boundary_no_vertical": (PP, "d = M[1:, :] != M[:-1, :]     # vertical neighbours differ",
                             "d = np.zeros_like(M[1:, :], bool)"),
    "frequency_last_map_only": (PP, "count += b", "count = b.astype(np.int64)"),
    "gradient_no_half": (PP, "gx = 0.5 * (right - left)", "gx = (right - left)"),
    "gradient_wraps_border": (PP, "right = f[:, np.minimum(xs + 1, W - 1), :]",
                              "right = f[:, (xs + 1) % W, :]"),
    "contour_not_normalised": (PP, "return (g / m).astype(np.float32)", "return g.astype(np.float32)"),
}
PY_WHERE = {PM: ["tests/test_oracle_metrics.py"], PP: ["tests/test_oracle_maps.py"]}


@pytest.mark.parametrize("name", sorted(PY_MUTATIONS))
def test_python_mutation_is_caught(name, tmp_path):
    fname, old, new = PY_MUTATIONS[name]
    work = tmp_path / "oracle"
    shutil.copytree(ORACLE, work, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = (work / fname).read_text()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    (work / fname).write_text(src.replace(old, new))
    env = dict(os.environ, SCALP_ORACLE_COPY_ROOT=str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PY_WHERE[fname]], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, (
        f"planted mistake '{name}' survived the pins:\n{r.stdout[-2000:]}")


def test_python_copy_is_the_one_tested(tmp_path):
    """The harness really swaps the package: an unmodified copy passes and a
    copy whose module raises on import fails."""
    work = tmp_path / "oracle"
    shutil.copytree(ORACLE, work, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    (work / PP).write_text((work / PP).read_text() + "\nraise ImportError('planted')\n")
    env = dict(os.environ, SCALP_ORACLE_COPY_ROOT=str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_maps.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0 and "planted" in r.stdout + r.stderr
