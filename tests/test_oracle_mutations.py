"""The oracle's pins catch plausible mistakes.

Each case copies the oracle to a temporary directory, plants one mistake in the
copy (a dropped term, a wrong sign, index or divisor, a transposed operand),
and checks that the oracle pin tests fail on it.  Nothing outside the temporary
copy is modified.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["test_oracle_dft.py", "test_oracle_variance.py", "test_oracle_update.py", "test_oracle_rng.py",
             "test_oracle_learned.py", "test_oracle_multiblock.py", "test_oracle_dst.py",
             "test_oracle_degenerate.py", "test_oracle_morph.py"]

MUTANTS = [
    ("enkf.py", "sum(axis=0) / (N - 1)", "sum(axis=0) / N"),
    ("enkf.py", "0.0, c_hat / safe)", "0.0, R_spec / safe)"),
    ("enkf.py", "(d_hat[None] + e_hat - u_hat)", "(d_hat[None] - e_hat - u_hat)"),
    ("enkf.py", "(a + 1j * b) / np.sqrt(2.0))", "(a + 1j * b))"),
    ("enkf.py", "np.where(mirrored, np.conj(zk), zk)", "zk"),
    ("enkf.py", "np.where(mirrored, ny - ky, ky)", "ky"),
    ("enkf.py", "if k % 2 == 0 else (words[2], words[3])", "if True else None"),
    ("enkf.py", "dev = ens - ens.mean(axis=0, keepdims=True)\n    c = np.empty", "dev = ens\n    c = np.empty"),
    ("enkf.py", "(x[:, None] - x[None, :]) % nx]", "(x[None, :] - x[:, None]) % nx]"),
    ("dft.py", "ang = (2.0 * np.pi / m)", "ang = (-2.0 * np.pi / m)"),
    ("dft.py", "np.conj(S[..., ky, nx - kx])", "S[..., ky, nx - kx]"),
    ("dft.py", "u @ wx_re + 1j * (u @ wx_im)", "u @ wx_re - 1j * (u @ wx_im)"),
    ("dft.py", "ky = (-np.arange(ny)) % ny", "ky = np.arange(ny)"),
    ("dft.py", "(dft_matrix(ny, +1) @ full @ dft_matrix(nx, +1))", "(dft_matrix(ny, -1) @ full @ dft_matrix(nx, +1))"),
    ("philox.py", "hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1", "hi1 ^ x[1] ^ k1, lo1, hi0 ^ x[3] ^ k0"),
    ("philox.py", "np.sqrt(-2.0 * np.log(u1))", "np.sqrt(-1.0 * np.log(u1))"),
    ("philox.py", "ang = 2.0 * np.pi * u2", "ang = np.pi * u2"),
    ("enkf.py", "cov = c_hat if lam is None else np.asarray(lam, dtype=np.float64)", "cov = c_hat"),
    ("multiblock.py", "(dj * np.conj(d1)).sum(axis=0)", "(np.conj(dj) * d1).sum(axis=0)"),
    ("multiblock.py", "out_hat[:, j] = u_hat[:, j] + G[None] * innov", "out_hat[:, j] = u_hat[:, 0] + G[None] * innov"),
    ("multiblock.py", "np.roll(a, (-hy, -hx), axis=(1, 2)) * b", "np.roll(a, (hy, hx), axis=(1, 2)) * b"),
    ("multiblock.py", "G = np.where(den < tiny, 0.0, cj1 / np.where(den < tiny, 1.0, den))",
     "G = np.where(den < tiny, 0.0, cj1 / np.where(den < tiny, 1.0, c11))"),
    ("dst.py", "    S[n - 1] /= np.sqrt(2.0)\n", "\n"),
    ("dst.py", "(2 * j + 1) * (k + 1) / (2 * n)", "(2 * j + 1) * k / (2 * n)"),
    ("dst.py", "((rel - rel.mean(axis=0)) ** 2).sum(axis=0) / (N - 1)", "((rel - rel.mean(axis=0)) ** 2).sum(axis=0) / N"),
    ("dst.py", "return dst2_matrix(ny).T @ s @ dst2_matrix(nx)", "return dst2_matrix(ny) @ s @ dst2_matrix(nx).T"),
    ("learned.py", "full[:, kx] = c_half[ky, nx - kx]", "full[:, kx] = c_half[:, nx - kx]"),
    ("learned.py", "dy, dx = j // 5 - 2, j % 5 - 2", "dx, dy = j // 5 - 2, j % 5 - 2"),
    ("learned.py", "np.log(full / mu + EPS)", "np.log(full + EPS)"),
    ("learned.py", "np.minimum(ky, ny - ky)", "ky + 0 * np.minimum(ky, ny - ky)"),
    ("learned.py", "+ lsb) >> np.uint64(16)", ") >> np.uint64(16)"),
    ("learned.py", "h = np.maximum(h @ W + b, 0.0)", "h = np.maximum(h @ W.T + b, 0.0)"),
    ("learned.py", "return mu * np.exp(y), mu", "return np.exp(y), mu"),
    ("learned.py", "K = spectral_gain(lam, R_spec, tiny)", "K = spectral_gain(c_hat, R_spec, tiny)"),
    ("learned.py", "if not (MU_MIN <= mu <= MU_MAX):", "if False:"),
    ("enkf.py", "s = u_hat - u_hat[0:1]", "s = u_hat"),
    ("enkf.py", "safe = np.where(den < tiny, 1.0, den)\n    return np.where(den < tiny, 0.0, c_hat / safe)",
     "return c_hat / den"),
    # centring either factor suffices (the other's deviations sum to zero), so
    # the plausible mistake is forgetting both
    ("multiblock.py", "dj = sj - sj.mean(axis=0, keepdims=True)\n    d1 = s1 - s1.mean(axis=0, keepdims=True)",
     "dj = sj\n    d1 = s1"),
    ("morph.py", "upd = upd + G[None] * innov[:, o]", "upd = upd + G[None] * innov[:, 0]"),
    ("morph.py", "cjo = cross_spectrum(u_hat[:, j], u_hat[:, o])", "cjo = cross_spectrum(u_hat[:, o], u_hat[:, j])"),
    ("morph.py", "z[:, o] = _noise(seed, N, ny, nx, o)", "z[:, o] = _noise(seed, N, ny, nx, 0)"),
    ("enkf.py", "np.where(nyq_sc, b, a) + 0j", "a + 0j"),
    ("morph.py", "G = np.where(den[o] < tiny, 0.0, cjo / np.where(den[o] < tiny, 1.0, den[o]))",
     "G = np.where(den[0] < tiny, 0.0, cjo / np.where(den[0] < tiny, 1.0, den[0]))"),
    ("morph.py", "if a != b and a < K and b < K:", "if False:"),
]


@pytest.mark.slow
@pytest.mark.parametrize("fname,before,after", MUTANTS, ids=[f"{m[0]}:{m[2][:24]}" for m in MUTANTS])
def test_pin_suite_catches_mutant(tmp_path, fname, before, after):
    for sub in ("oracle", "tests"):
        shutil.copytree(os.path.join(ROOT, sub), tmp_path / sub,
                        ignore=shutil.ignore_patterns("__pycache__", "test_oracle_mutations.py"))
    pkg = tmp_path / "paper_1001_1588_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1001_1588_amd", "twin.py"), pkg / "twin.py")
    (pkg / "__init__.py").write_text("")
    target = tmp_path / "oracle" / fname
    src = target.read_text()
    assert before in src, "mutation anchor not found; update the mutant list"
    target.write_text(src.replace(before, after, 1))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          *[os.path.join("tests", t) for t in PIN_TESTS]],
                         cwd=tmp_path, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, "mutant survived the oracle pin tests:\n" + res.stdout[-2000:]
