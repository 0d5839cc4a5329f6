"""The oracle's pins catch plausible mistakes: each planted mistake below, built into a copy of
oracle.c, makes at least one pin of tests/test_oracle_pins.py fail (CPU only).

A mistake that no pin catches would mean the oracle could carry it unnoticed; the list covers the
hop (projector sign, link placement, neighbour offset, time boundary), the Dirac matrices, the
clover (leaf sum and normalisation) and the clover inverse."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MUTATIONS = {
    "forward projector 1 + g instead of 1 - g": (
        "double pm = dir == 0 ? -1.0 : +1.0;", "double pm = dir == 0 ? +1.0 : -1.0;"),
    "backward link not conjugated": (
        "mat3_dagger(link(U, V, mu, j), u);", "memcpy(u, link(U, V, mu, j), sizeof u);"),
    "forward link taken at the neighbour": (
        "memcpy(u, link(U, V, mu, i), sizeof u);", "memcpy(u, link(U, V, mu, j), sizeof u);"),
    "neighbour two sites away": (
        "d[mu] = (d[mu] + step + L[mu]) % L[mu];", "d[mu] = (d[mu] + 2 * step + 2 * L[mu]) % L[mu];"),
    "antiperiodic sign missing on the forward t hop": (
        "if (dir == 0 && c[3] == L[3] - 1) sign = -sign;", ""),
    "gamma_1 entry with the wrong sign": (
        "g[0][3] = I; g[1][2] = I; g[2][1] = -I; g[3][0] = -I;", "g[0][3] = I; g[1][2] = I; g[2][1] = I; g[3][0] = -I;"),
    "field strength normalised by 1/4": (
        "F[k] = (Q[k] - Qd[k]) / 8.0;", "F[k] = (Q[k] - Qd[k]) / 4.0;"),
    "third clover leaf dropped": (
        "mat3_mul(t1, link(U, V, nu, s_mn), leaf);\n    for (int k = 0; k < 9; k++) Q[k] += leaf[k];",
        "mat3_mul(t1, link(U, V, nu, s_mn), leaf);"),
    "Gauss-Jordan elimination adds instead of subtracting": (
        "for (int k = 0; k < 12; k++) a[r][k] -= f * a[col][k];",
        "for (int k = 0; k < 12; k++) a[r][k] += f * a[col][k];"),
}


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    old, new = MUTATIONS[name]
    with open(os.path.join(ROOT, "oracle", "oracle.c")) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(mutant), "-lm"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, QCDW_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x", "-q",
                        "-p", "no:cacheprovider", "-k", "not dense_lu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"no pin failed for the planted mistake '{name}':\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout


FGMRES_MUTATIONS = {
    "Arnoldi coefficient without the conjugate": ("H[i, j] = np.vdot(V[i], w)", "H[i, j] = np.dot(V[i], w)"),
    "last Gram-Schmidt projection dropped": ("for i in range(j + 1):", "for i in range(j):"),
    "update built from the Arnoldi vectors instead of the preconditioned ones": (
        "x = x + np.stack(Z[:k], axis=1) @ y", "x = x + np.stack(V[:k], axis=1) @ y"),
    "restart keeps the old residual": ("        r = bf - op(x)\n        beta = float(np.linalg.norm(r))\n    return",
                                       "    return"),
    "least-squares right-hand side not scaled by beta": ("e1[0] = beta", "e1[0] = 1.0"),
}


@pytest.mark.parametrize("name", list(FGMRES_MUTATIONS))
def test_planted_fgmres_mistake_fails_a_pin(monkeypatch, name):
    """Each planted mistake in a copy of oracle/fgmres.py makes at least one FGMRES pin fail."""
    from tests import test_oracle_fgmres as pins

    old, new = FGMRES_MUTATIONS[name]
    with open(os.path.join(ROOT, "oracle", "fgmres.py")) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    ns = {"__name__": "fgmres_mutant"}
    exec(compile(src.replace(old, new), "fgmres_mutant.py", "exec"), ns)
    monkeypatch.setattr(pins, "fgmres", ns["fgmres"])
    checks = [pins.test_full_cycle_solves_a_dense_system_exactly,
              *[(lambda k=k: pins.test_minimal_residual_over_the_krylov_space(k)) for k in (1, 3, 6)],
              pins.test_flexible_arnoldi_relation_with_a_changing_preconditioner,
              pins.test_exact_inverse_as_preconditioner_converges_in_one_step,
              pins.test_restarts_reach_the_tolerance]
    failed = 0
    for check in checks:
        try:
            check()
        except Exception:  # an assertion, or the mutant breaking outright
            failed += 1
    assert failed > 0, f"no FGMRES pin failed for the planted mistake '{name}'"


MG_MUTATIONS = {
    "restriction without the complex conjugate": ("prod = (np.conj(w) * r).sum(axis=2)", "prod = (w * r).sum(axis=2)"),
    "chirality split by the wrong spins": ("chi_of_spin = np.array([0, 0, 1, 1])", "chi_of_spin = np.array([0, 1, 0, 1])"),
    "Gram-Schmidt without normalisation": ("cols[k] = w / nrm", "cols[k] = w"),
    "Gram-Schmidt projection on the raw vectors": ("w = w - np.vdot(cols[j], w) * cols[j]",
                                                   "w = w - np.vdot(vecs[j][m], w) * cols[j]"),
    "coarse sites numbered with y fastest": (
        "idx = ((cx[:, 3] * Lc[2] + cx[:, 2]) * Lc[1] + cx[:, 1]) * Lc[0] + cx[:, 0]",
        "idx = ((cx[:, 3] * Lc[2] + cx[:, 2]) * Lc[0] + cx[:, 0]) * Lc[1] + cx[:, 1]"),
    "smoothing step with the wrong sign": ("z = z + (np.vdot(w, r) / np.vdot(w, w)) * r",
                                           "z = z - (np.vdot(w, r) / np.vdot(w, w)) * r"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", list(MG_MUTATIONS))
def test_planted_multigrid_mistake_fails_a_pin(monkeypatch, name):
    """Each planted mistake in a copy of oracle/multigrid.py makes at least one multigrid pin fail."""
    import types

    from tests import test_oracle_multigrid as pins

    old, new = MG_MUTATIONS[name]
    with open(os.path.join(ROOT, "oracle", "multigrid.py")) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    mod = types.ModuleType("multigrid_mutant")
    exec(compile(src.replace(old, new), "multigrid_mutant.py", "exec"), mod.__dict__)
    monkeypatch.setattr(pins, "mg", mod)
    checks = [pins.test_block_index_enumerates_blocks,
              pins.test_block_gram_schmidt_matches_qr_and_spans_the_vectors,
              pins.test_single_site_aggregates_with_a_full_basis_reproduce_M,
              lambda: pins.test_free_field_coarse_operator_closed_form((2, 2, 2, 2)),
              lambda: pins.test_free_field_coarse_operator_closed_form((2, 1, 2, 4)),
              pins.test_coarse_operator_gamma5_hermitian_and_nearest_neighbour,
              pins.test_coarse_operator_gauge_invariant,
              pins.test_two_level_fgmres_beats_plain_gmres]
    failed = 0
    for check in checks:
        try:
            check()
        except Exception:
            failed += 1
    assert failed > 0, f"no multigrid pin failed for the planted mistake '{name}'"


FORCE_MUTATIONS = {
    "variation multiplied from the right": ("Up[mu, i] = Uf[mu, i] + 1j * T[a] @ Uf[mu, i]",
                                           "Up[mu, i] = Uf[mu, i] + 1j * Uf[mu, i] @ T[a]"),
    "variation without the factor i": ("Up[mu, i] = Uf[mu, i] + 1j * T[a] @ Uf[mu, i]",
                                       "Up[mu, i] = Uf[mu, i] + T[a] @ Uf[mu, i]"),
    "imaginary part of the bilinear": ("H[mu, i] += 2.0 * np.vdot(Y, d).real * T[a]",
                                       "H[mu, i] += 2.0 * np.vdot(Y, d).imag * T[a]"),
    "factor 2 of the real part dropped": ("H[mu, i] += 2.0 * np.vdot(Y, d).real * T[a]",
                                          "H[mu, i] += np.vdot(Y, d).real * T[a]"),
    "a generator with the wrong normalisation": ("lam[7] = np.diag([1, 1, -2]) / np.sqrt(3)",
                                                 "lam[7] = np.diag([1, 1, -2]) / 3"),
}


@pytest.mark.parametrize("name", list(FORCE_MUTATIONS))
def test_planted_force_mistake_fails_a_pin(monkeypatch, name):
    """Each planted mistake in a copy of oracle/force.py makes at least one force pin fail."""
    import types

    from tests import test_oracle_force as pins

    old, new = FORCE_MUTATIONS[name]
    with open(os.path.join(ROOT, "oracle", "force.py")) as f:
        src = f.read()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    mod = types.ModuleType("force_mutant")
    exec(compile(src.replace(old, new), "force_mutant.py", "exec"), mod.__dict__)
    monkeypatch.setattr(pins, "of", mod)
    checks = [pins.test_generators_normalised,
              lambda: pins.test_force_matches_group_finite_difference(1),
              pins.test_two_flavour_hmc_force,
              pins.test_force_gauge_covariant_and_hermitian_traceless]
    failed = 0
    for check in checks:
        try:
            check()
        except Exception:
            failed += 1
    assert failed > 0, f"no force pin failed for the planted mistake '{name}'"
