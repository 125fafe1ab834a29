"""The factored kernel's running-sum moments, pinned on the CPU.

The kernel forms the lag moments of a 64-sample block, M_q = sum_r (r - 31.5)^q z_r, from
iterated running sums (S_0 += z_r, then S_k += S_(k-1) per sample, which end as
S_k = sum_r C(63 - r + k, k) z_r) and a basis change A worked out at compile time,
M_q = sum_(k<=q) A[q][k] S_k. This test compiles the kernel source's own compile-time
basis (the host-evaluable `moment_basis`) with g++ and checks it against the basis derived
here in exact rational arithmetic, and checks the recurrence plus basis change against the
moments summed directly, in FP64, for Q = 1 .. 6.
"""
import os
import re
import shutil
import subprocess
from fractions import Fraction
from math import comb

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2508_06672_amd", "csrc", "k_direct_fact.hip")
QMAX = 6
FB = 64


def kernel_basis(tmp_path):
    """A[q][k] for Q = 1 .. QMAX as the kernel's compile-time code computes it (floats)."""
    src = open(SRC).read()
    start = src.index("template <int Q>\nstruct MomentBasis {")
    end = src.index("template <int Q>\nstruct MomentBasisTable")
    prog = ["#include <cstdio>", f"constexpr int kFB = {FB};", src[start:end]]
    prog.append("template <int Q> void dump() { constexpr MomentBasis<Q> m = moment_basis<Q>();"
                " for (int q = 0; q < Q; ++q) for (int k = 0; k < Q; ++k)"
                " std::printf(\"%d %d %d %.9g\\n\", Q, q, k, (double)m.a[q][k]); }")
    prog.append("int main() { " + " ".join(f"dump<{q}>();" for q in range(1, QMAX + 1)) + " return 0; }")
    cpp = tmp_path / "basis.cpp"
    exe = tmp_path / "basis"
    cpp.write_text("\n".join(prog))
    subprocess.run(["g++", "-std=c++17", "-O1", str(cpp), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    A = {Q: np.zeros((Q, Q)) for Q in range(1, QMAX + 1)}
    for line in out.splitlines():
        Q, q, k, v = line.split()
        A[int(Q)][int(q), int(k)] = float(v)
    return A


def exact_basis(Q):
    """(c - u)^q = sum_k A[q][k] C(u + k, k), c = 31.5, solved in exact rationals: both sides
    are polynomials in u, C(u + k, k) has degree k and leading coefficient 1/k!."""
    def poly_mul(a, b):
        out = [Fraction(0)] * (len(a) + len(b) - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(b):
                out[i + j] += x * y
        return out

    P = []
    for k in range(Q):
        p = [Fraction(1)]
        for i in range(1, k + 1):
            p = poly_mul(p, [Fraction(i), Fraction(1)])
        fact = Fraction(1)
        for i in range(1, k + 1):
            fact *= i
        P.append([x / fact for x in p])
    c = Fraction(FB - 1, 2)
    A = [[Fraction(0)] * Q for _ in range(Q)]
    for q in range(Q):
        t = [Fraction(1)]
        for _ in range(q):
            t = poly_mul(t, [c, Fraction(-1)])
        t = t + [Fraction(0)] * (Q - len(t))
        for d in range(q, -1, -1):
            w = t[d] / P[d][d]
            A[q][d] = w
            for e in range(d + 1):
                t[e] -= w * P[d][e]
        assert all(x == 0 for x in t)
    return A


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_kernel_basis_matches_exact_rationals(tmp_path):
    A = kernel_basis(tmp_path)
    for Q in range(1, QMAX + 1):
        E = exact_basis(Q)
        for q in range(Q):
            for k in range(Q):
                e = float(E[q][k])
                if k > q:
                    assert A[Q][q, k] == 0.0 and e == 0.0, (Q, q, k)
                else:
                    # the kernel keeps A in FP32: within half an FP32 unit of the exact value
                    assert abs(A[Q][q, k] - e) <= 2.0 ** -24 * abs(e), (Q, q, k, A[Q][q, k], e)
        # the diagonal is (-1)^q q!, integral and exact
        for q in range(Q):
            assert A[Q][q, q] == (-1) ** q * float(np.prod(range(1, q + 1)))


def test_running_sums_give_the_centred_moments():
    """The recurrence in the kernel's order, then the exact basis, equals the moments summed
    directly (FP64, random complex samples, and a block whose samples are all equal)."""
    rng = np.random.default_rng(5)
    r = np.arange(FB) - 0.5 * (FB - 1)
    for Q in range(1, QMAX + 1):
        A = np.array([[float(x) for x in row] for row in exact_basis(Q)])
        for z in (rng.standard_normal(FB) + 1j * rng.standard_normal(FB), np.full(FB, 0.3 - 0.7j)):
            S = np.zeros(Q, complex)
            for n in range(FB):
                S[0] += z[n]
                for k in range(1, Q):
                    S[k] += S[k - 1]
            # closed form of each level
            for k in range(Q):
                w = np.array([comb(FB - 1 - n + k, k) for n in range(FB)], float)
                assert abs(S[k] - np.sum(w * z)) <= 1e-9 * np.sum(w * np.abs(z))
            M = A @ S
            direct = np.array([np.sum(r ** q * z) for q in range(Q)])
            scale = np.array([np.sum(np.abs(r) ** q * np.abs(z)) for q in range(Q)])
            assert np.all(np.abs(M - direct) <= 1e-9 * np.maximum(scale, 1.0) * 32.0 ** np.arange(Q)), Q
