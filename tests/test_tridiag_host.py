"""Host build of the tridiagonal eigen-solver the error control runs on the
device (csrc/kry_tridiag.h, compiled here with g++): eigenvalues and the
first and last eigenvector rows against LAPACK (numpy.linalg.eigh), through
the quantity the bound uses, (e^{tT})_{m,1} = sum_i q_{m,i} q_{1,i} e^{theta_i t}."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_01583_amd", "csrc")

HARNESS = r"""
#include <cstdio>
#include <vector>
#include "kry_tridiag.h"
int main() {
    int nm;
    if (scanf("%d", &nm) != 1) return 1;
    for (int t = 0; t < nm; ++t) {
        int m;
        if (scanf("%d", &m) != 1) return 1;
        std::vector<double> d(m), e(m), q1(m), qm(m);
        for (int i = 0; i < m; ++i) if (scanf("%lf", &d[i]) != 1) return 1;
        for (int i = 0; i < m - 1; ++i) if (scanf("%lf", &e[i]) != 1) return 1;
        const bool ok = kry::tridiag_eig_rows(m, d.data(), e.data(), q1.data(), qm.data());
        printf("%d %d\n", m, ok ? 1 : 0);
        for (int i = 0; i < m; ++i) printf("%.17g %.17g %.17g\n", d[i], q1[i], qm[i]);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_tridiag_eigen_rows_against_lapack(tmp_path):
    src = tmp_path / "tri.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "tri"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    rng = np.random.default_rng(5)
    cases = []
    for m in (1, 2, 3, 7, 40, 200, 700):
        cases.append((rng.normal(size=m), rng.uniform(0.1, 2.0, size=m - 1)))
    # a Lanczos-like matrix of a stiff operator: diagonal in [-1200, 0], tight clusters
    m = 300
    d = -np.sort(rng.uniform(0, 1200, size=m))
    d[100:110] = d[100] + 1e-9 * np.arange(10)
    cases.append((d, rng.uniform(1e-3, 300, size=m - 1)))
    text = f"{len(cases)}\n" + "".join(
        f"{len(d)}\n" + " ".join(repr(float(x)) for x in d) + "\n" + " ".join(repr(float(x)) for x in e) + "\n"
        for d, e in cases)
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    pos = 0
    for d, e in cases:
        m, ok = map(int, out[pos].split())
        pos += 1
        rows = np.array([[float(x) for x in out[pos + i].split()] for i in range(m)])
        pos += m
        assert ok == 1 and m == len(d)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        w, Q = np.linalg.eigh(T)
        scale = np.abs(T).max()
        assert np.abs(np.sort(rows[:, 0]) - w).max() <= 1e-13 * m * scale
        # the orthogonal rows: |q1| = |qm| = 1
        assert abs(np.sum(rows[:, 1] ** 2) - 1) < 1e-12 and abs(np.sum(rows[:, 2] ** 2) - 1) < 1e-12
        for t in (1e-3, 0.1, 1.0):
            tt = t / max(scale, 1.0)
            want = np.sum(Q[-1] * Q[0] * np.exp(w * tt))
            got = np.sum(rows[:, 2] * rows[:, 1] * np.exp(rows[:, 0] * tt))
            assert abs(got - want) <= 1e-12 * m
