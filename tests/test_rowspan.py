"""Host logic of the pruned darkfield FFT passes (Eq. 11-13 chain): the row
ranges they run over. A signed row span becomes a cyclic range of FFT-order
rows, rounded up to whole row-pass workgroups; the pass that forms P_hat runs
over the shortest cyclic range holding this image's rows and the previous
image's (which it clears). Checked against brute force over random cases,
with g++ on the CPU; skipped when no host compiler is available."""

import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def run_cases(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path_factory.mktemp("rowspan") / "rowspan_check"
    subprocess.run([gxx, "-std=c++17", "-O1", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined",
                    os.path.join(ROOT, "tests", "native", "rowspan_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, text=True)

    def run(lines):
        r = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True,
                           text=True, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        return [tuple(map(int, l.split())) for l in r.stdout.split("\n") if l.strip()]

    return run


def _rows(y0, n, grid):
    return {(y0 + i) % grid for i in range(n)}


def _rounded(rows, grid, group):
    return min(grid, max(group, -(-rows // group) * group))


def test_spans_become_rounded_cyclic_ranges(run_cases):
    rng = np.random.default_rng(0)
    cases, want = [], []
    for _ in range(400):
        grid = int(rng.choice([64, 128, 256, 512]))
        group = 4 * 256 // grid  # rows per workgroup of the FP64 row passes
        lo = int(rng.integers(-grid // 2, grid // 2))
        hi = int(rng.integers(lo - 1, min(lo + grid, grid // 2)))
        cases.append(f"s {grid} {group} {lo} {hi}")
        want.append((lo % grid, _rounded(hi - lo + 1, grid, group)))
    got = run_cases(cases)
    assert got == want
    for (y0, n), c in zip(got, cases):
        grid, group, lo, hi = map(int, c.split()[1:])
        assert {ky % grid for ky in range(lo, hi + 1)} <= _rows(y0, n, grid)
        assert n % group == 0 or n == grid


def test_hull_is_the_shortest_cover_of_both_ranges(run_cases):
    rng = np.random.default_rng(1)
    cases, ab = [], []
    for _ in range(600):
        grid = int(rng.choice([64, 128, 256]))
        group = 4 * 256 // grid
        a = (int(rng.integers(0, grid)), int(rng.integers(1, grid + 1)))
        b = (int(rng.integers(0, grid)), int(rng.integers(1, grid + 1)))
        cases.append(f"h {grid} {group} {a[0]} {a[1]} {b[0]} {b[1]}")
        ab.append((grid, group, a, b))
    got = run_cases(cases)
    for (y0, n), (grid, group, a, b) in zip(got, ab):
        need = _rows(*a, grid) | _rows(*b, grid)
        assert need <= _rows(y0, n, grid)
        # the shortest cyclic run covering both: the grid minus the longest
        # cyclic run of rows that neither range holds
        free = [y not in need for y in range(grid)] * 2
        gap = run = 0
        for f in free:
            run = run + 1 if f else 0
            gap = max(gap, min(run, grid))
        assert n == _rounded(grid - gap, grid, group)


def test_first_image_covers_every_row(run_cases):
    """Before the first image the previous range is the whole grid: the pass
    clears every row an earlier call left behind."""
    got = run_cases([f"h 256 4 0 256 {y0} {n}" for y0, n in [(0, 4), (200, 100), (97, 60)]])
    assert all(r == (0, 256) for r in got)
