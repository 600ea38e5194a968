"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/sdbie.h declares, and rejects invalid arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdbie.h")


@pytest.fixture(scope="module")
def L():
    from paper_2110_10749_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2110_10749_amd import build
        build.build()
    return binding.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 12, names
    for n in names:
        assert hasattr(L, n), f"{n} declared in sdbie.h but not exported"


def test_header_constants_match_the_binding():
    from paper_2110_10749_amd import binding as B
    src = open(HEADER).read()
    defs = dict(re.findall(r"^#define\s+(SDBIE_[A-Z0-9_]+)\s+(\S+)", src, flags=re.M))
    assert int(defs["SDBIE_SYM_LAPLACE"]) == B.SYM_LAPLACE and int(defs["SDBIE_SYM_STOKES"]) == B.SYM_STOKES
    assert int(defs["SDBIE_SYM_LAPLACE_F64"]) == B.SYM_LAPLACE_F64
    assert int(defs["SDBIE_SYM_STOKES_F64"]) == B.SYM_STOKES_F64 and int(defs["SDBIE_SYM_ALL"]) == B.SYM_ALL
    assert B.SYM_ALL == B.SYM_LAPLACE | B.SYM_STOKES | B.SYM_LAPLACE_F64 | B.SYM_STOKES_F64
    m = re.search(r"^#define\s+SDBIE_SYM_DEFAULT\s+\((.*)\)\s*$", open(HEADER).read(), flags=re.M)
    default = 0
    for name in m.group(1).split("|"):
        default |= int(defs[name.strip()])
    assert default == B.SYM_DEFAULT
    assert int(defs["SDBIE_NOALLOC_MAX_NODES"]) == B.NOALLOC_MAX_NODES


def test_abi_version_and_default_opts(L):
    from paper_2110_10749_amd import binding
    assert L.sdbie_abi_version() == 4
    o = binding.default_opts()
    assert o.tol_gmres == 1e-10 and o.tol_ddm == 1e-8 and o.theta == 0.5
    assert o.restart == 50 and o.outer == 1 and o.slip == 0 and o.prec == 0
    assert o.tol_mixed == 1e-4 and o.mixed_mode == 2 and o.relax_outer == 1 and o.local_solver == 0 and o.recycle == 1


def test_workspace_bytes(L):
    from paper_2110_10749_amd import binding
    a = binding.workspace_bytes(4302, 50)
    b = binding.workspace_bytes(68166, 50)
    assert 0 < a < b
    assert binding.workspace_bytes(68166, 10) < b
    assert binding.workspace_bytes(0, 50) == 0
    assert binding.workspace_bytes(100, 0) == 0
    assert binding.workspace_bytes(100, 1000) > 0 and binding.workspace_bytes(100, 1001) == 0


@pytest.mark.parametrize("n,m,splits", [(4096, 50, 64), (68166, 50, 16), (68166, 1000, 16), (351866, 50, 8),
                                         (524288, 50, 8), (524289, 50, 8), (1 << 23, 50, 8)])
def test_workspace_formula_in_header(L, n, m, splits):
    # the header's estimate (120 m + 1185 + 96 S) n + (n/256)^2 * q, q = 3471
    # up to 524288 nodes (masks and symmetric lists), 2 above (masks only),
    # within 1%
    from paper_2110_10749_amd import binding
    nt = (n + 255) // 256
    q = 3471 if n <= 524288 else 2
    est = (120 * m + 1185 + 96 * splits) * n + q * nt * nt
    assert abs(est / binding.workspace_bytes(n, m) - 1.0) < 0.01


def test_invalid_arguments_are_rejected_on_the_host(L):
    from paper_2110_10749_amd import binding as B
    # null plan pointer / null surface
    assert L.sdbie_plan_create(None, None, 50, None, 0, None) == B.ERR_ARG
    h = ctypes.c_void_p()
    assert L.sdbie_plan_create(ctypes.byref(h), None, 50, None, 0, None) == B.ERR_ARG
    assert b"null surface" in L.sdbie_last_error()
    surf = B.Surface(10, 1, 1, 1, 0.1)
    # bad delta
    bad = B.Surface(10, 1, 1, 1, -1.0)
    assert L.sdbie_plan_create(ctypes.byref(h), ctypes.byref(bad), 50, None, 0, None) == B.ERR_ARG
    for d in (1e-16, 2e15, float("inf"), float("nan")):  # outside [1e-15, 1e15]
        bad = B.Surface(10, 1, 1, 1, d)
        assert L.sdbie_plan_create(ctypes.byref(h), ctypes.byref(bad), 50, None, 0, None) == B.ERR_ARG
    # n out of range
    bad = B.Surface(0, 1, 1, 1, 0.1)
    assert L.sdbie_plan_create(ctypes.byref(h), ctypes.byref(bad), 50, None, 0, None) == B.ERR_ARG
    # workspace missing, misaligned, too small
    assert L.sdbie_plan_create(ctypes.byref(h), ctypes.byref(surf), 50, None, 0, None) == B.ERR_WORKSPACE
    assert L.sdbie_plan_create(ctypes.byref(h), ctypes.byref(surf), 50, ctypes.c_void_p(4096 + 8), 10**9, None) == B.ERR_WORKSPACE
    assert L.sdbie_plan_create(ctypes.byref(h), ctypes.byref(surf), 50, ctypes.c_void_p(4096), 16, None) == B.ERR_WORKSPACE
    assert b"too small" in L.sdbie_last_error()
    # null plan on every entry point
    assert L.laplace_layer_apply(None, 0, None, None, 0, None) == B.ERR_ARG
    assert L.stokes_layer_apply(None, 1.0, 0, None, None, 0, None) == B.ERR_ARG
    prm = B.Params(1.0, 1.0, 0.0)
    U = (ctypes.c_double * 3)(0, 0, 1)
    assert L.darcy_solve(None, ctypes.byref(prm), None, None, None, None, None) == B.ERR_ARG
    assert L.stokes_solve(None, ctypes.byref(prm), U, None, None, None, None, None, None) == B.ERR_ARG
    d = (ctypes.c_double * 3)()
    assert L.ddm_solve(None, ctypes.byref(prm), U, None, None, None, d, None, None, None) == B.ERR_ARG
    assert L.sdbie_plan_n(None) == -1
    assert L.sdbie_plan_set_symmetric(None, 1) == B.ERR_ARG


def _match(a, b):
    """Largest distance from each value of a to the nearest unused value of b."""
    b = list(b)
    worst = 0.0
    for z in a:
        j = min(range(len(b)), key=lambda i: abs(b[i] - z))
        worst = max(worst, abs(b[j] - z))
        b.pop(j)
    return worst


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (7, 3), (40, 4), (150, 5)])
def test_hessenberg_eigenvalues_match_lapack(L, n, seed):
    # the host step of the D-N spectrum: the Francis QR iteration on an upper
    # Hessenberg matrix against LAPACK's general eigenvalue routine
    import numpy as np
    from paper_2110_10749_amd import binding as B
    rng = np.random.default_rng(seed)
    H = np.triu(rng.normal(size=(n, n)), -1)
    got = np.array(B.hessenberg_eigenvalues(H))
    ref = np.linalg.eigvals(H)
    assert _match(got, ref) < 1e-10 * max(1.0, np.abs(H).sum())


def test_hessenberg_eigenvalues_of_arnoldi_like_matrices(L):
    # the Hessenberg matrix of Arnoldi on a matrix with clustered real
    # eigenvalues (multiplets, as the D-N map has on a sphere) and a complex pair
    import numpy as np
    from paper_2110_10749_amd import binding as B
    rng = np.random.default_rng(7)
    lam = np.concatenate([np.full(3, -1 / 3) + 1e-6 * rng.normal(size=3),
                          np.full(5, -0.104) + 1e-6 * rng.normal(size=5), rng.uniform(-0.05, 0.0, 60)])
    n = lam.size + 2
    D = np.zeros((n, n))
    D[np.arange(lam.size), np.arange(lam.size)] = lam
    D[-2:, -2:] = [[0.2, 0.3], [-0.3, 0.2]]
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ D @ Q.T
    m = 50
    V = np.zeros((n, m + 1))
    Hm = np.zeros((m + 1, m))
    v = rng.normal(size=n)
    V[:, 0] = v / np.linalg.norm(v)
    for k in range(m):
        w = A @ V[:, k]
        for _ in range(2):
            h = V[:, :k + 1].T @ w
            w -= V[:, :k + 1] @ h
            Hm[:k + 1, k] += h
        Hm[k + 1, k] = np.linalg.norm(w)
        V[:, k + 1] = w / Hm[k + 1, k]
    got = np.array(B.hessenberg_eigenvalues(Hm[:m, :m]))
    assert _match(got, np.linalg.eigvals(Hm[:m, :m])) < 1e-12


def test_hessenberg_eigenvalues_rejects_bad_arguments(L):
    from paper_2110_10749_amd import binding as B
    assert L.sdbie_hessenberg_eigenvalues(0, None, None, None) == B.ERR_ARG


def test_noalloc_entry_point_rejects_arguments_on_the_host(L):
    # the allocation-free layer sum checks its arguments before any device work
    from paper_2110_10749_amd import binding as B
    assert L.stokes_layer_apply_noalloc(None, 1.0, 0, None, None, 0, None) == B.ERR_ARG
    assert b"null surface" in L.sdbie_last_error()
    big = B.Surface(B.NOALLOC_MAX_NODES + 1, 4096, 4096, 4096, 0.1)
    assert L.stokes_layer_apply_noalloc(ctypes.byref(big), 1.0, 0, None, None, 0, None) == B.ERR_ARG
    assert b"allocation-free" in L.sdbie_last_error()
    bad = B.Surface(100, 4096, 4096, 4096, -1.0)
    assert L.stokes_layer_apply_noalloc(ctypes.byref(bad), 1.0, 0, None, None, 0, None) == B.ERR_ARG


def test_hessenberg_eigenvalues_with_exact_multiplets(L):
    # Arnoldi on a symmetric matrix whose eigenvalues repeat exactly in the
    # multiplets of the D-N map on a sphere (lambda_n of the free-slip closed
    # form, 2n + 1 times each): the Hessenberg matrix then holds copies of one
    # eigenvalue in separate blocks, and a double shift from the trailing 2x2
    # block alone annihilates the first column of the QR step (the iteration
    # used to stall on such matrices); against LAPACK
    import numpy as np
    from paper_2110_10749_amd import binding as B
    rng = np.random.default_rng(0)
    lam = []
    for n in range(1, 40):
        lam += [-(n + 1) * (2 * n + 1) / (2 * n * (n + 2) * (2 * n * n + 1))] * (2 * n + 1)
    lam = np.array(lam[:1200])
    Q, _ = np.linalg.qr(rng.normal(size=(lam.size, lam.size)))
    A = (Q * lam) @ Q.T
    m = 120
    V = np.zeros((lam.size, m + 1))
    Hm = np.zeros((m + 1, m))
    v = rng.normal(size=lam.size)
    V[:, 0] = v / np.linalg.norm(v)
    for k in range(m):
        w = A @ V[:, k]
        for _ in range(2):
            h = V[:, :k + 1].T @ w
            w -= V[:, :k + 1] @ h
            Hm[:k + 1, k] += h
        Hm[k + 1, k] = np.linalg.norm(w)
        V[:, k + 1] = w / Hm[k + 1, k]
    got = np.array(B.hessenberg_eigenvalues(Hm[:m, :m]))
    ref = np.linalg.eigvals(Hm[:m, :m])
    assert _match(got, ref) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed,K,noise", [(0, 1.0, 1e-7), (4, 1e-2, 3e-7), (11, 1e-4, 1e-8)])
def test_hessenberg_eigenvalues_of_inexact_arnoldi(L, seed, K, noise):
    # Arnoldi whose products carry a relative error (as with float pair sums in
    # the local solves): the multiplets of the D-N map split into clusters of
    # eigenvalues a few ulps to 1e-8 apart, and a double-shift step whose first
    # column is formed from the sum and product of the shifts cancels to noise
    # on them (the iteration stalled on these matrices); against LAPACK
    import numpy as np
    from paper_2110_10749_amd import binding as B
    rng = np.random.default_rng(seed)
    lam = []
    for n in range(1, 60):
        lam += [-(n + 1) * (2 * n + 1) / (2 * n * (n + 2) * (2 * n * n + 1)) / K] * (2 * n + 1)
    lam = np.array(lam[:2000])
    Q, _ = np.linalg.qr(rng.normal(size=(lam.size, lam.size)))
    A = (Q * lam) @ Q.T
    m = 240
    V = np.zeros((lam.size, m + 1))
    Hm = np.zeros((m + 1, m))
    v = rng.normal(size=lam.size)
    V[:, 0] = v / np.linalg.norm(v)
    for k in range(m):
        w = A @ V[:, k]
        w += noise * np.linalg.norm(w) * rng.normal(size=w.size) / np.sqrt(w.size)
        for _ in range(2):
            h = V[:, :k + 1].T @ w
            w -= V[:, :k + 1] @ h
            Hm[:k + 1, k] += h
        Hm[k + 1, k] = np.linalg.norm(w)
        V[:, k + 1] = w / Hm[k + 1, k]
    got = np.array(B.hessenberg_eigenvalues(Hm[:m, :m]))
    ref = np.linalg.eigvals(Hm[:m, :m])
    assert _match(got, ref) < 1e-12 * np.max(np.abs(ref))
