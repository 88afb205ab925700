"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is compiled a second time, with ``-fsanitize=address,undefined``
and no recovery, into a temporary directory, and a child Python process (with
the ASan runtime preloaded, as a ctypes-loaded library needs) drives every
entry point through the oracle's own wrappers: rasterisation in every mode,
Kalman steps, field initialisations, sweeps with and without a source term,
the relaxation to a certificate, the index matrix, descents (also cut short)
and the rubber band, on small and ragged grids and on one grid large enough
for the OpenMP branches.  Any out-of-bounds access, use after free or
undefined operation aborts the child with the sanitizer's report.  OpenMP
runs are not checked for races here: ThreadSanitizer needs an instrumented
OpenMP runtime.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "twg_oracle.c")


def _runtime(name):
    gcc = shutil.which("gcc")
    if gcc is None:
        return None
    path = subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


CHILD = textwrap.dedent(
    """
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    from paper_1903_07441_amd import scenarios
    oracle._LIB = LIB
    oracle._lib = None

    def exercise(sc):
        nx, ny = sc["nx"], sc["ny"]
        cls, ring = oracle.rasterize(sc)
        cls2, _ = oracle.rasterize(sc, method="allpairs", border_walls=False)
        static = np.zeros((ny, nx), np.uint8)
        static[ny // 2, :: 3] = 1
        oracle.rasterize(sc, static_occ=static)
        n = len(sc["rad"])
        cov = np.tile(np.diag([0.25, 0.25, 0.1, 0.1]).reshape(16), (n, 1))
        oracle.rasterize_modes(sc, ring_mode=1, heading=(0.6, 0.8), per_object=True, kappa=1.0, cov=cov)
        oracle.ring_map(nx, ny, sc["robot"], sc["W"])
        for init in (oracle.INIT_HALF, oracle.INIT_ZERO, oracle.INIT_LINEAR):
            oracle.field_init(cls, mode=init, goal=sc["goal"])
        psi, info = oracle.relax(cls, tol=1e-9, tol_cert=1e-6, goal=sc["goal"])
        f = np.linspace(-1e-3, 1e-3, nx * ny).reshape(ny, nx)
        oracle.residual(cls, psi, f)
        oracle.residual_field(cls, psi, f)
        oracle.sor_sweep(cls, psi, 1.5, f)
        oracle.jacobi_step(cls, psi)
        oracle.gs_lex_step(cls, psi)
        oracle.relax(cls, psi=psi, init=oracle.INIT_KEEP, f=f, tol=1e-8, max_sweeps=200)
        oracle.index_matrix(cls, psi)
        st, path = oracle.descend(cls, psi, sc["robot"])
        oracle.descend(cls, psi, sc["robot"], cap=1)
        oracle.goal_reachable(cls, sc["robot"])
        if len(path) >= 3:
            oracle.rubber_band(cls, psi, path, k=1.0, iters=4)

    for nx, ny, n_obs, seed in ((3, 2, 0, 1), (5, 5, 1, 2), (17, 9, 3, 3), (40, 30, 8, 4), (33, 64, 12, 5)):
        exercise(scenarios.custom(nx, ny, n_obs, rad=(1.0, 4.0), seed=seed, W=3))

    x = np.array([5.0, 6.0, 0.5, -0.25])
    P = np.diag([0.25, 0.25, 0.1, 0.1]).reshape(16)
    Q = np.eye(4).reshape(16) * 1e-3
    x2, P2 = oracle.kalman_predict_steps(x, P, 1.0, 7, Q=Q)
    oracle.kalman_update(x2, P2, np.array([5.5, 5.5]), np.eye(2) * 0.1)
    oracle.pos_cov(P, 3.0)
    oracle.inflated_radius(2.0, P, 3.0, 1.0, 8)
    oracle.ring_ellipse(7, -3, 0.6, 0.8, 8)
    oracle.predict_mean(x[:2], x[2:], 2.5)

    # above 65536 cells the sweeps, residuals and maps take their OpenMP branches
    big = scenarios.custom(300, 240, 20, rad=(2.0, 6.0), seed=6)
    cls, _ = oracle.rasterize(big)
    psi = oracle.field_init(cls, mode=oracle.INIT_HALF, goal=big["goal"])
    for _ in range(3):
        psi = oracle.sor_sweep(cls, psi, 1.9)
    oracle.residual(cls, psi)
    oracle.residual_field(cls, psi)
    oracle.index_matrix(cls, psi)
    print("SANITIZERS-CLEAN", flush=True)
    """
)


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None or _runtime("libubsan.so") is None:
        pytest.skip("gcc or its sanitizer runtimes are not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    SRC, "-o", lib, "-lm"], check=True)
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    script = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "SANITIZERS-CLEAN" in r.stdout, (r.stdout[-2000:], r.stderr[-6000:])
