"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the printed
text of the paper (lookup tables, the memory table, quoted factors), hand
derivations of tiny cases, closed forms (Lucas' theorem, the triangle's
binary-as-ternary form), library routines (2-D convolution, a symmetric
eigensolver) and brute force.
"""
import math
import os

import numpy as np
import pytest
from scipy.signal import convolve2d

import fractals as FR

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def frac(oracle, name, r):
    s, offs = FR.ALL[name]
    return oracle.Fractal(s, offs, r)


# ---------------------------------------------------------------------------
# construction, volume, compact order
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,rmax", [("triangle", 9), ("triangle_paper", 7), ("carpet", 4), ("vicsek", 5)])
def test_volume_and_distinct_cells(oracle_lib, name, rmax):
    """Eq. V: the level-r fractal has k^r cells, all distinct, inside [0, s^r)^2."""
    for r in range(0, rmax + 1):
        F = frac(oracle_lib, name, r)
        xy = F.order()
        assert xy.shape == (F.k ** r, 2)
        assert xy.min() >= 0 and xy.max() < F.n
        assert len({(int(a), int(b)) for a, b in xy}) == F.N


def test_triangle_worked_example_golden(oracle_lib):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "triangle_order_r2.txt")) if l[0] != "#"]
    want = np.array([[int(x), int(y)] for _, x, y in rows])
    assert (frac(oracle_lib, "triangle", 2).order() == want).all()


@pytest.mark.parametrize("r", range(0, 9))
def test_triangle_is_lucas_set(oracle_lib, r):
    """Lucas' theorem: (x,y) is in the level-r Sierpinski triangle iff x & y == 0,
    and there are exactly 3^r such points in the 2^r box."""
    F = frac(oracle_lib, "triangle", r)
    got = {(int(a), int(b)) for a, b in F.order()}
    n = 2 ** r
    want = {(x, y) for y in range(n) for x in range(n) if x & y == 0}
    assert got == want and len(want) == 3 ** r


def test_paper_triangle_orientation(oracle_lib):
    """Section 'Revisiting lambda': tau(0)=(0,0), tau(1)=(0,1), tau(2)=(1,1) gives the
    mirror image (x subset-of-bits y) of the x & y == 0 triangle."""
    for r in range(0, 8):
        F = frac(oracle_lib, "triangle_paper", r)
        got = {(int(a), int(b)) for a, b in F.order()}
        n = 2 ** r
        assert got == {(x, y) for y in range(n) for x in range(n) if x & ~y == 0}


# ---------------------------------------------------------------------------
# lambda and nu
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,r", [("triangle", 10), ("triangle_paper", 6), ("carpet", 4), ("vicsek", 5)])
def test_lambda_formula_matches_replication(oracle_lib, name, r):
    F = frac(oracle_lib, name, r)
    assert (F.lam(np.arange(F.N)) == F.order()).all()


@pytest.mark.parametrize("name,r", [("triangle", 9), ("carpet", 4), ("vicsek", 5)])
def test_nu_matches_dense_inverse_with_ring(oracle_lib, name, r):
    """nu (top-down) equals the inverse of the replication order on every point of
    [-1, n]^2: members map to their index, holes and the outer ring to HOLE."""
    F = frac(oracle_lib, name, r)
    dense = F.dense_inverse()
    ring = np.full((F.n + 2, F.n + 2), -1, dtype=np.int64)
    ring[1:-1, 1:-1] = dense
    ys, xs = np.mgrid[-1:F.n + 1, -1:F.n + 1]
    got = F.nu(np.stack([xs.ravel(), ys.ravel()], 1)).reshape(ring.shape)
    assert (got == ring).all()
    # nu o lambda = id and every hole is rejected
    assert (F.nu(F.lam(np.arange(F.N))) == np.arange(F.N)).all()
    assert (got == -1).sum() == (F.n + 2) ** 2 - F.N


def b3(v: int) -> int:
    """Read the binary digits of v as ternary digits."""
    return int(bin(v)[2:], 3)


def test_triangle_binary_as_ternary_closed_form(oracle_lib):
    """x & y == 0 triangle: nu(x, y) = B3(x) + 2 B3(y) (replica 1 carries x's bit,
    replica 2 carries y's bit at each level)."""
    F = frac(oracle_lib, "triangle", 12)
    rng = np.random.default_rng(5)
    xs = rng.integers(0, F.n, 20000)
    ys = rng.integers(0, F.n, 20000)
    got = F.nu(np.stack([xs, ys], 1))
    want = np.array([b3(x) + 2 * b3(y) if x & y == 0 else -1 for x, y in zip(xs.tolist(), ys.tolist())])
    assert (got == want).all()
    assert (want >= 0).sum() > 100


def test_paper_triangle_hash(oracle_lib):
    """Section 'Case study': for the paper's triangle the lookup table H_nu[(0,0)]=0,
    H_nu[(0,1)]=1, H_nu[(1,1)]=2 equals the hash theta_x + theta_y on replica digit
    pairs, so nu(x,y) = sum_mu (theta_x + theta_y) 3^(mu-1) on every member."""
    F = frac(oracle_lib, "triangle_paper", 10)
    xy = F.order().astype(np.int64)
    want = np.zeros(F.N, dtype=np.int64)
    for mu in range(1, F.r + 1):
        tx = (xy[:, 0] >> (mu - 1)) & 1
        ty = (xy[:, 1] >> (mu - 1)) & 1
        want += (tx + ty) * 3 ** (mu - 1)
    assert (F.nu(xy) == want).all()


def beta_paper(wx, wy, mu, k):
    """The paper's beta equation on a 2-D compact coordinate (wx, wy)."""
    num = wx * (mu % 2) + wy * ((mu + 1) % 2)
    return (num // k ** (math.ceil(mu / 2) - 1)) % k


@pytest.mark.parametrize("name,r", [("triangle", 5), ("triangle", 6), ("carpet", 3), ("vicsek", 4)])
def test_paper_beta_formula_is_interleaved_linear_index(oracle_lib, name, r):
    """Section 'Compacting NBB Fractals' + the beta equation: over the compact
    rectangle (width k^ceil(r/2), height k^floor(r/2)) the paper's lambda is a
    bijection onto the fractal, and equals the oracle's lambda of the linear index
    whose digit mu-1 is beta_mu (odd levels from wx, even levels from wy)."""
    F = frac(oracle_lib, name, r)
    s, k = F.s, F.k
    W, H = k ** math.ceil(r / 2), k ** (r // 2)
    offs = np.array(F.offsets)
    pts, lin = [], []
    for wy in range(H):
        for wx in range(W):
            x = y = c = 0
            for mu in range(1, r + 1):
                b = beta_paper(wx, wy, mu, k)
                x += offs[b, 0] * s ** (mu - 1)
                y += offs[b, 1] * s ** (mu - 1)
                c += b * k ** (mu - 1)
            pts.append((x, y))
            lin.append(c)
    assert len(set(pts)) == F.N == W * H
    assert set(pts) == {(int(a), int(b)) for a, b in F.order()}
    assert (F.lam(np.array(lin)) == np.array(pts)).all()


def test_paper_nu_axis_filters_as_printed_transpose(oracle_lib):
    """Reading of the nu equations: with theta_mu taken as the level-mu digit pair,
    Delta^nu_mu = k^floor((mu-1)/2) and H_nu = replica index, the filters as printed
    (f_x = (mu-1) mod 2, f_y = mu mod 2) return the transposed compact coordinate;
    swapping them inverts the paper's lambda.  We use the inverse."""
    F = frac(oracle_lib, "triangle", 5)
    k, r = F.k, F.r
    for wy in range(k ** (r // 2)):
        for wx in range(k ** math.ceil(r / 2)):
            c = sum(beta_paper(wx, wy, mu, k) * k ** (mu - 1) for mu in range(1, r + 1))
            x, y = F.lam([c])[0]
            nx_p = ny_p = nx_s = ny_s = 0
            for mu in range(1, r + 1):
                tx, ty = (x >> (mu - 1)) & 1, (y >> (mu - 1)) & 1
                h = F.offsets.index((int(tx), int(ty)))
                d = k ** ((mu - 1) // 2)
                nx_p += d * h * ((mu - 1) % 2)
                ny_p += d * h * (mu % 2)
                nx_s += d * h * (mu % 2)
                ny_s += d * h * ((mu - 1) % 2)
            assert (nx_s, ny_s) == (wx, wy)
            assert (nx_p, ny_p) == (wy, wx)


# ---------------------------------------------------------------------------
# memory reduction factor (closed form of Eq. V against the printed table)
# ---------------------------------------------------------------------------

def test_memory_table_r16(oracle_lib):
    """Table at r=16: block size rho leaves r_b = 16 - log2(rho) compact levels with an
    expanded rho x rho micro-fractal each, 4 bytes per cell.  MRF = n^2 / (3^r_b rho^2)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "memory_table_r16.txt")) if l[0] != "#"]
    n = 2 ** 16
    for rho, bb, sq, mrf in rows:
        rho = int(rho)
        rb = 16 - int(math.log2(rho))
        F = frac(oracle_lib, "triangle", min(rb, 8))
        V = F.k ** rb  # Eq. V (its replication count is checked above for r <= 9)
        assert F.N == 3 ** F.r
        bb_gib = n * n * 4 / 2 ** 30
        sq_gib = V * rho * rho * 4 / 2 ** 30
        assert bb_gib == float(bb)
        assert abs(sq_gib - float(sq)) <= 0.01
        assert round(n * n / (V * rho * rho), 1) == float(mrf)


def test_r20_memory_claims():
    """Section 'Memory Reduction Factor': r=20 BB needs 4096 GB (4 B/cell), Squeeze
    ~13 to ~55 GB over rho=1..32, MRF ~315."""
    n = 2 ** 20
    assert n * n * 4 / 2 ** 30 == 4096
    lo = 3 ** 20 * 4 / 2 ** 30
    hi = 3 ** 15 * 32 * 32 * 4 / 2 ** 30
    assert round(lo) == 13 and round(hi) == 55
    assert round((4 / 3) ** 20) == 315


def test_theoretical_mrf_plot_values():
    """Section 'Theoretical Memory Reduction Factor': at n = 2^16 the plot reads
    close to 400x (Vicsek), 105x (triangle), 3.4x (carpet).  MRF = n^2 / k^r with
    r = log_s n; read from a plot, so compared within 10%."""
    n = 2.0 ** 16
    for s, k, quoted in ((3, 5, 400.0), (2, 3, 105.0), (3, 8, 3.4)):
        r = math.log(n, s)
        assert abs(n * n / k ** r / quoted - 1) < 0.10


# ---------------------------------------------------------------------------
# Life on the fractal
# ---------------------------------------------------------------------------

KERNEL8 = np.array([[1, 1, 1], [1, 0, 1], [1, 1, 1]])


def life_by_convolution(member, state):
    cnt = convolve2d(state * member, KERNEL8, mode="same", boundary="fill", fillvalue=0)
    out = ((cnt == 3) | ((state == 1) & (cnt == 2))).astype(np.uint8)
    return out * member


@pytest.mark.parametrize("name,r", [("triangle", 7), ("triangle_paper", 6), ("carpet", 4), ("vicsek", 4)])
@pytest.mark.parametrize("seed", FR.SEEDS[:2])
def test_life_matches_convolution(oracle_lib, name, r, seed):
    """Masked B3/S23 (holes neither simulated nor counted) on the expanded grid and
    through lambda/nu, against a 2-D convolution of the masked grid."""
    F = frac(oracle_lib, name, r)
    member = F.member()
    grid = F.fill_expanded(seed, 0.5)
    assert (grid <= member).all()
    want = life_by_convolution(member.astype(np.int64), grid.astype(np.int64))
    assert (oracle_lib.life_expanded(member, grid) == want).all()
    xy = F.order()
    compact = grid[xy[:, 1], xy[:, 0]]
    assert (F.fill_compact(seed, 0.5) == compact).all()
    assert (F.life_compact(compact) == want[xy[:, 1], xy[:, 0]]).all()
    # several steps through the neighbour table
    g = grid.astype(np.int64)
    for _ in range(4):
        g = life_by_convolution(member.astype(np.int64), g)
    assert (F.life_steps(compact, 4) == g[xy[:, 1], xy[:, 0]]).all()


def test_life_tiny_cases(oracle_lib):
    F0 = frac(oracle_lib, "triangle", 0)
    assert F0.life_compact(np.array([1], np.uint8)).tolist() == [0]  # lone cell dies
    F1 = frac(oracle_lib, "triangle", 1)
    assert F1.life_compact(np.ones(3, np.uint8)).tolist() == [1, 1, 1]  # still life
    for dead in range(3):
        st = np.ones(3, np.uint8)
        st[dead] = 0
        assert F1.life_compact(st).tolist() == [0, 0, 0]


@pytest.mark.parametrize("r,alive", [(2, 5), (3, 13), (10, 26245)])
def test_all_alive_counts(oracle_lib, r, alive):
    F = frac(oracle_lib, "triangle", r)
    out = F.life_compact(np.ones(F.N, np.uint8))
    assert out.sum() == alive
    if r <= 6:
        member = F.member().astype(np.int64)
        assert life_by_convolution(member, member).sum() == alive


def test_triangle_degree_histogram_r10(oracle_lib):
    F = frac(oracle_lib, "triangle", 10)
    deg = (F.neighbour_table() >= 0).sum(1)
    hist = dict(zip(*np.unique(deg, return_counts=True)))
    assert {int(a): int(b) for a, b in hist.items()} == {2: 3, 3: 26242, 4: 26244, 5: 6560}
    assert deg.sum() == 2 * 108254
    member = F.member().astype(np.int64)
    conv = convolve2d(member, KERNEL8, mode="same") * member
    assert conv.sum() == deg.sum()


@pytest.mark.parametrize("name,r,t", [("triangle", 7, 3), ("triangle", 8, 6), ("carpet", 4, 4), ("vicsek", 5, 5)])
def test_light_cone_matches_full_simulation(oracle_lib, name, r, t):
    F = frac(oracle_lib, name, r)
    seed, p = 99, 0.3
    full = F.life_steps(F.fill_compact(seed, p), t)
    rng = np.random.default_rng(1)
    cs = rng.choice(F.N, size=min(F.N, 3000), replace=False)
    xy = F.lam(cs)
    assert (F.light_cone(seed, p, xy, t) == full[cs]).all()


@pytest.mark.parametrize("name,r,t", [("triangle", 7, 5), ("triangle_paper", 6, 3), ("carpet", 4, 4),
                                      ("vicsek", 4, 6)])
def test_life_windows_match_convolution(oracle_lib, name, r, t):
    """Rectangles of the t-step state (the window form of the light cone) against t
    steps of a 2-D convolution of the whole masked grid: rectangles inside the box,
    straddling its edges and corners, partly and wholly outside it, and the whole box."""
    F = frac(oracle_lib, name, r)
    seed, p = 7, 0.45
    member = F.member().astype(np.int64)
    g = F.fill_expanded(seed, p).astype(np.int64)
    for _ in range(t):
        g = life_by_convolution(member, g)
    n = F.n
    pad = np.zeros((n + 40, n + 40), np.int64)
    pad[20:20 + n, 20:20 + n] = g
    rects = [(0, 0, n, n), (3, 5, 17, 9), (-6, -4, 13, 11), (n - 7, n - 3, 12, 9), (n - 5, -2, 9, 6),
             (-3, n - 4, 8, 10), (n + 2, n + 1, 5, 4), (n // 3, n // 2, 1, 1), (-8, 4, 6, 5)]
    for (x0, y0, w, h) in rects:
        got = F.life_windows(seed, p, [(x0, y0)], w, h, t)[0]
        want = pad[20 + y0:20 + y0 + h, 20 + x0:20 + x0 + w]
        assert got.shape == want.shape and (got == want).all(), (name, r, x0, y0, w, h)
    # several rectangles of one size in one call
    corners = [(1, 2), (n - 9, 0), (0, n - 9)]
    got = F.life_windows(seed, p, corners, 9, 9, t)
    for q, (x0, y0) in enumerate(corners):
        assert (got[q] == pad[20 + y0:29 + y0, 20 + x0:29 + x0]).all()


# ---------------------------------------------------------------------------
# seeded inputs
# ---------------------------------------------------------------------------

def test_splitmix64_published_vector(oracle_lib):
    """Reference output of SplitMix64 seeded with 0 (first three draws)."""
    assert oracle_lib.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert oracle_lib.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert oracle_lib.splitmix64(0, 2) == 0x06C45D188009454F


def test_bernoulli_thresholds_and_density(oracle_lib):
    assert oracle_lib.threshold24(0.5) == 8388608
    assert oracle_lib.threshold24(0.3) == 5033164
    F = frac(oracle_lib, "triangle", 11)
    for p in (0.5, 0.3):
        m = F.fill_compact(2201, p).mean()
        assert abs(m - p) < 4 * math.sqrt(p * (1 - p) / F.N)


def test_uniform_fill_is_24bit_grid(oracle_lib):
    F = frac(oracle_lib, "carpet", 3)
    u = F.fill_uniform_compact(7)
    assert u.min() >= 0 and u.max() < 1
    assert (u * 2 ** 24 == np.floor(u * 2 ** 24)).all()
    assert abs(u.mean() - 0.5) < 0.02


# ---------------------------------------------------------------------------
# diffusion (binary64): spectral solution from a library eigensolver
# ---------------------------------------------------------------------------

def moore_laplacian(member):
    ys, xs = np.nonzero(member)
    idx = -np.ones(member.shape, dtype=np.int64)
    idx[ys, xs] = np.arange(len(xs))
    n = member.shape[0]
    A = np.zeros((len(xs), len(xs)))
    for i, (y, x) in enumerate(zip(ys, xs)):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx or dy) and 0 <= y + dy < n and 0 <= x + dx < n and idx[y + dy, x + dx] >= 0:
                    A[i, idx[y + dy, x + dx]] = 1
    return np.diag(A.sum(1)) - A, idx


@pytest.mark.parametrize("name,r", [("triangle", 1), ("carpet", 1), ("vicsek", 1), ("triangle", 4), ("carpet", 2)])
def test_diffusion_matches_spectral_solution(oracle_lib, name, r):
    """u_{t+1} = (I - a L) u_t with L the Moore-graph Laplacian of the fractal: after t
    steps u_t = V diag((1 - a lam_i)^t) V^T u_0 (eigh is the library routine)."""
    F = frac(oracle_lib, name, r)
    a, t = 0.1, 25
    member = F.member()
    L, idx = moore_laplacian(member)
    lam, V = np.linalg.eigh(L)
    xy = F.order()
    perm = idx[xy[:, 1], xy[:, 0]]  # compact index -> row of L
    u0 = F.fill_uniform_compact(3)
    v0 = np.empty(F.N)
    v0[perm] = u0
    want_rows = V @ (((1 - a * lam) ** t) * (V.T @ v0))
    got = F.diffuse_steps(u0, a, t)
    assert np.allclose(got, want_rows[perm], rtol=0, atol=1e-12)
    assert abs(got.sum() - u0.sum()) < 1e-12 * F.N
    if name == "triangle" and r == 1:
        assert np.allclose(sorted(lam), [0, 3, 3])
    if name == "carpet" and r == 1:
        assert np.allclose(sorted(lam), [0, 3 - math.sqrt(3), 3 - math.sqrt(3), 2, 4,
                                         3 + math.sqrt(3), 3 + math.sqrt(3), 6])


def test_diffusion_single_step_forms_agree(oracle_lib):
    F = frac(oracle_lib, "carpet", 3)
    u = F.fill_uniform_compact(11)
    assert np.array_equal(F.diffuse_compact(u, 0.1), F.diffuse_steps(u, 0.1, 1))
    ones = np.full(F.N, 0.375)
    assert (F.diffuse_compact(ones, 0.1) == 0.375).all()


@pytest.mark.parametrize("name,r,t", [("carpet", 4, 3), ("carpet", 5, 7), ("vicsek", 5, 4), ("triangle", 7, 5)])
def test_diffusion_light_cone_matches_full_field(oracle_lib, name, r, t):
    F = frac(oracle_lib, name, r)
    a, seed = 0.1, 21
    full = F.diffuse_steps(F.fill_uniform_compact(seed), a, t)
    rng = np.random.default_rng(3)
    cs = rng.choice(F.N, size=min(F.N, 2000), replace=False)
    got = F.diffuse_cone(seed, a, F.lam(cs), t)
    assert np.allclose(got, full[cs], rtol=0, atol=1e-13)
