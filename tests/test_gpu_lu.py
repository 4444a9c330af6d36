"""The stage-matrix factorisation alone (LU with partial pivoting of
M = d I - J, Sec. 2.3), through chem_lu, against the oracle's LU.

Both launches' routines are checked: the team launches' (one wavefront per
matrix for N <= 64, a work-group of four wavefronts for 64 < N <= 128; rows
stay in their lanes and the pivot is the largest |M_ik| over the unused rows,
ties to the lowest row of M) and the one-cell-per-thread launches' (explicit
row swaps, ties to the lowest current position, as the oracle and LAPACK).

Bar: the permutation is index work and must agree exactly wherever it is
unique - where the oracle's runner-up in every column is more than 1e-12
(relative) below the pivot; with an exact or near tie either choice is a valid
partial pivot, which the bound |L| <= 1 checks.  The factors are floating
point: the GPU divides by multiplying with the pivot's reciprocal and
contracts a - l u into one FMA, so they differ from the oracle's by
rounding.  Gaussian elimination with partial pivoting guarantees a backward
error |L U - P M| <= gamma_N |L||U| (gamma_N = N eps / (1 - N eps)), which
each GPU factorisation must meet with a factor 2 to spare; on well-scaled
random matrices every factor entry is also within 8 N eps |L||U| of the
oracle's (the L part divided by |U_kk|), and on the Jacobians - condition
numbers up to 1e22, where single tiny multipliers lose all relative
accuracy to cancellation in either code - each row of (L diag(U), U) within
1e-8 of that row's largest |L||U| entry.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2205_05681_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = np.finfo(float).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def chem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_05681_amd import chem as C
    C.lib()
    return C


def gpu_lu(chem, As, d, launch):
    """chem_lu on the stack As (n, N, N): the factors of M = d I - A (the
    library forms M itself), their order perm and the status, per matrix."""
    n, N, _ = As.shape
    A = np.ascontiguousarray(As.reshape(n, N * N).T)
    At = torch.from_numpy(A).cuda()
    F, perm, status = chem.lu(At, d, launch)
    torch.cuda.synchronize()
    F = F.cpu().numpy().T.reshape(n, N, N)
    return F, perm.cpu().numpy().T.astype(np.int64), status.cpu().numpy()


def split(F):
    N = F.shape[0]
    return np.tril(F, -1) + np.eye(N), np.triu(F)


def check_one(F, perm, M, ref, exact_factors, label):
    """One GPU factorisation against the oracle's (F, perm, status, margin)."""
    N = M.shape[0]
    Fo, po, so, margin = ref
    assert so == 0, label
    assert np.array_equal(np.sort(perm), np.arange(N)), label
    L, U = split(F)
    assert np.abs(L).max() <= 1.0, label                      # a valid partial pivot at every step
    absLU = np.abs(L) @ np.abs(U)
    gamma = N * EPS / (1 - N * EPS)
    assert np.all(np.abs(L @ U - M[perm]) <= 2 * gamma * absLU + 1e-300), label
    if margin <= 1e-12 and not np.array_equal(perm, po):
        return "tie"                                           # several valid pivot orders
    assert np.array_equal(perm, po), (label, margin)
    Lo, Uo = split(Fo)
    absLUo = np.abs(Lo) @ np.abs(Uo)
    if exact_factors:
        low = np.tril(np.ones((N, N), bool), -1)
        scale = np.where(low, absLUo / np.abs(np.diag(Uo))[None, :], absLUo)
        assert np.all(np.abs(F - Fo) <= 8 * N * EPS * scale + 1e-300), label
    else:
        low = np.tril(np.ones((N, N), bool), -1)
        G = np.where(low, F * np.diag(U)[None, :], F)
        Go = np.where(low, Fo * np.diag(Uo)[None, :], Fo)
        assert np.all(np.abs(G - Go) <= 1e-8 * absLUo.max(axis=1, keepdims=True)), label
    return "same"


def random_matrices(rng, n, N):
    """n matrices of order N: normal entries with rows and columns scaled by
    10^U(-2, 2), a quarter of the off-diagonal entries zero (the Jacobians'
    sparsity), and in every third one M_00 = 0 with M_10 and M_01 nonzero (a
    forced interchange, structurally nonsingular)."""
    Ms = rng.normal(size=(n, N, N))
    Ms *= 10.0 ** rng.uniform(-2, 2, size=(n, N, 1)) * 10.0 ** rng.uniform(-2, 2, size=(n, 1, N))
    off = ~np.eye(N, dtype=bool)[None]
    Ms[(rng.random(size=Ms.shape) < 0.25) & off] = 0.0
    if N > 1:
        for c in range(0, n, 3):
            Ms[c, 0, 0] = 0.0
            Ms[c, 1, 0] = 1.0 + rng.random()
            Ms[c, 0, 1] = 1.0 + rng.random()
    return Ms


@pytest.mark.parametrize("launch,N", [("team", 1), ("team", 2), ("team", 16), ("team", 31), ("team", 54),
                                      ("team", 56), ("team", 64), ("team", 65), ("team", 112), ("team", 128),
                                      ("thread", 1), ("thread", 54), ("thread", 112), ("thread", 200)])
def test_lu_random_matrices(chem, launch, N):
    """67 matrices (two 64-thread groups in the thread launch, the second
    ragged) per size: every kernel the team launches are compiled for (16,
    32, 48, 56 and 64 rows; four wavefronts up to 128), with and without
    padding rows, and the thread launch up to N = 200."""
    rng = np.random.default_rng(1000 + N)
    n = 67
    Ms = random_matrices(rng, n, N)
    say("case: chem_lu %s N=%d, %d random matrices" % (launch, N, n))
    # d = 0: A = -M, so M = 0 I - A is M exactly
    F, perm, status = gpu_lu(chem, -Ms, 0.0, launch)
    assert np.all(status == 0)
    kinds = [check_one(F[c], perm[c], Ms[c], oracle.lu(Ms[c]), True, (launch, N, c)) for c in range(n)]
    assert kinds.count("same") == n


@pytest.mark.parametrize("name", ["ch4", "large"])
def test_lu_jacobians(chem, mech_dir, name):
    """M = I/(h gamma) - J with the oracle's Jacobians at 24 mixing-layer
    states (the hottest twelve and twelve more), h from 1e-10 s to 1e-4 s
    (gamma of ROS4): the matrices the integrator factors, in both launches."""
    path, m = synth.mechanism_file(name, mech_dir)
    o = oracle.Oracle(path)
    T, P, Y = synth.states_mixing(m, 4096, 204)
    idx = np.r_[np.argsort(-T)[:12], np.arange(12)]
    Js = []
    for c in idx:
        Js.append(o.jacobian(P[c], o.to_phi(T[c], P[c], Y[:, c])))
    Js = np.array(Js)
    N = Js.shape[1]
    gamma = oracle.method_table("ros4")["gamma"]
    for h in (1e-10, 1e-8, 1e-6, 1e-4):
        d = 1.0 / (h * gamma)
        Ms = np.array([(d * np.eye(N)) - J for J in Js])
        # the library forms M = d I - A itself: hand it J
        refs = [oracle.lu(Mc) for Mc in Ms]
        for launch in ("team", "thread"):
            say("case: chem_lu %s on %s Jacobians, N=%d, h=%g" % (launch, name, N, h))
            F, perm, status = gpu_lu(chem, Js, d, launch)
            assert np.all(status == 0)
            kinds = [check_one(F[c], perm[c], Ms[c], refs[c], False, (name, h, launch, c))
                     for c in range(len(idx))]
            say("  same order %d, tie resolved otherwise %d" % (kinds.count("same"), kinds.count("tie")))


def implicit_lu_order(M):
    """The team routine's pivot rule by brute force, on a matrix whose
    elimination is exact in binary (small integers, multipliers 1/2): the
    largest magnitude over the rows not yet used, ties to the lowest row."""
    A = M.astype(float).copy()
    N = A.shape[0]
    used = np.zeros(N, bool)
    order = []
    for k in range(N):
        cand = np.where(~used)[0]
        v = np.abs(A[cand, k])
        p = cand[np.flatnonzero(v == v.max())[0]]
        order.append(p)
        used[p] = True
        for r in np.where(~used)[0]:
            A[r, k:] -= (A[r, k] / A[p, k]) * A[p, k:]
    return np.array(order)


def tie_matrix(N, rows):
    """A 3 x 3 block on rows (r0, r1, r2) and columns 0..2 - r2 pivots
    column 0, after which rows r0 and r1 tie at 1 in column 1 - and unit rows
    covering columns 3..N-1 elsewhere.  With r0 = 0 < r1 < r2 the row swap of
    column 0 moves row 0 below row r1, so the two tie rules choose different
    rows."""
    r0, r1, r2 = rows
    M = np.zeros((N, N))
    M[r0, :3] = [1.0, 1.0, 1.0]
    M[r1, :3] = [0.0, 1.0, 3.0]
    M[r2, :3] = [2.0, 0.0, 1.0]
    others = [r for r in range(N) if r not in rows]
    for j, r in enumerate(others):
        M[r, 3 + j] = 1.0
    return M


@pytest.mark.parametrize("N,rows", [(54, (0, 1, 2)), (54, (0, 7, 40)), (112, (0, 70, 100)),
                                    (112, (0, 66, 5)), (128, (10, 67, 127))])
def test_lu_pivot_ties(chem, N, rows):
    """Exact ties after a row interchange: the team routine takes the lowest
    row of M (across both halves of the four-wavefront split), the thread
    routine the lowest current position, as the oracle; both factorisations
    reproduce M exactly.  Plus an exact tie in column 0, where the two rules
    agree."""
    M = tie_matrix(N, rows)
    T0 = np.eye(N)
    T0[[3, 9]] = 0.0
    T0[3, 0], T0[9, 0] = -4.0, 4.0              # column 0 tie between rows 3 and 9
    T0[3, 3], T0[9, 9] = 1.0, 1.0
    Ms = np.array([M, T0])
    say("case: chem_lu pivot ties, N=%d rows %s" % (N, rows))
    want_team = [implicit_lu_order(Mc) for Mc in Ms]
    want_thread = [oracle.lu(Mc)[1] for Mc in Ms]
    if rows[0] == 0 and rows[1] < rows[2]:
        assert not np.array_equal(want_team[0], want_thread[0])   # the case separates the rules
    assert want_team[1][0] == 3 and want_thread[1][0] == 3
    for launch, want in (("team", want_team), ("thread", want_thread)):
        F, perm, status = gpu_lu(chem, -Ms, 0.0, launch)
        assert np.all(status == 0)
        for c in range(2):
            assert np.array_equal(perm[c], want[c]), (launch, c)
            L, U = split(F[c])
            assert np.array_equal(L @ U, Ms[c][perm[c]]), (launch, c)


@pytest.mark.parametrize("launch,N", [("team", 54), ("team", 112), ("thread", 54)])
def test_lu_status_codes(chem, launch, N):
    """A zero column gives 1, NaN or an infinity in a pivot column 2, the first
    failure in column order; a zero row gives 1 at the last step; the good
    matrices of the same batch are unaffected."""
    rng = np.random.default_rng(77)
    Ms = random_matrices(rng, 8, N)
    Ms[1, :, 5] = 0.0                                # zero column
    Ms[2, 4, 7] = np.nan                             # NaN
    Ms[3, 9, 2] = np.inf                             # infinity
    Ms[4, :, 3] = 0.0                                # zero column before a NaN
    Ms[4, 6, 8] = np.nan
    Ms[5, 2, 3] = np.nan                             # NaN before a zero column
    Ms[5, :, 6] = 0.0
    Ms[6, N // 2, :] = 0.0                           # zero row
    say("case: chem_lu status codes, %s N=%d" % (launch, N))
    F, perm, status = gpu_lu(chem, -Ms, 0.0, launch)
    assert list(status) == [0, 1, 2, 2, 1, 2, 1, 0]
    for c in (0, 7):
        assert check_one(F[c], perm[c], Ms[c], oracle.lu(Ms[c]), True, (launch, N, c)) == "same"
    assert [oracle.lu(Mc)[2] for Mc in Ms] == list(status)


def test_lu_arguments(chem):
    """Argument errors come back as codes, before any launch."""
    from paper_2205_05681_amd.chem import ChemError
    A = torch.zeros((5, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        chem.lu(A, 1.0)                                  # not N*N rows
    A = torch.zeros((129 * 129, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(ChemError):
        chem.lu(A, 1.0, "team")                          # above the team routines' 128
    A = torch.zeros((4, 0), dtype=torch.float64, device="cuda")
    F, perm, status = chem.lu(A, 1.0)                    # an empty batch
    assert F.shape == (4, 0) and status.shape == (0,)
