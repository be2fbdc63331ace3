"""Hand-derived pins of the oracle's band operators: mixing of small, new and
vanishing cells (Sec. 2.3.2, applied after every Runge-Kutta sub-step), the
ghost-state extension that supplies a material's state outside its region
(Sec. 2.3.2, the ghost state of the interface Riemann problem) and the
level-set advection velocity v^n (Eq. local-advection).

Each case is a few cells whose result follows from the definition by hand:
the expected numbers below are written out (fractions, averages), not
recomputed with the oracle's formulas.  The readings pinned are:

* mixing: targets are the x, y and diagonal neighbours on the side of
  increasing phi^r, eligible with alpha_t >= alpha_mix and chi_t = r; weights
  g_x^2 alpha, g_y^2 alpha, |g_x g_y| alpha normalised to beta; a full
  exchange with one target leaves source and target at the same averaged
  conserved density U = (Q_s + Q_t)/(alpha_s + alpha_t) ("calculated
  according to the averaged values"), and target t receives the fraction
  beta_t of that exchange; without an eligible x/y/diagonal target the
  8-neighbour of largest alpha (ties: lower linear index) takes all; a
  vanishing source hands over all of its state, exactly; a source with no
  eligible neighbour at all (stranded) joins the cell's own material, or, if
  it is the cell's own material, the material of largest other alpha, to
  which the cell is then relabelled;
* extension: Jacobi sweeps from the upwind neighbours along increasing
  phi^r weighted by |g_x|, |g_y|, a value once set is kept, then sweeps of
  the mean of the valid neighbours; the band reaches 4 cells;
* velocity: 4 Jacobi sweeps from the neighbours towards smaller phi
  weighted by |g_x|, |g_y|, then the material's own velocity.

Every case is chosen so that a plausible slip (|g| for g^2, a dropped
diagonal target, no exact remainder, an upwind sign flip, Gauss-Seidel for
Jacobi, a mean over all 8 neighbours instead of the valid ones) changes an
asserted value.
"""
import numpy as np
import pytest

import oracle
import workloads as wl

RT = 1e-14


def cfg2(nx, ny, M=2, **kw):
    return wl.base_config(dim=2, nx=nx, ny=ny, n_mat=M, x0=0.0, x1=float(nx),
                          y0=0.0, y1=float(ny), gamma=[1.4] * M, pinf=[0.0] * M, **kw)


def cfg1(nx, M=2, **kw):
    return wl.base_config(dim=1, nx=nx, ny=1, n_mat=M, x0=0.0, x1=float(nx),
                          gamma=[1.4] * M, pinf=[0.0] * M, **kw)


def close(a, b, rt=RT):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.allclose(a, b, rtol=rt, atol=rt * max(1.0, np.abs(b).max()))


def pair_exchange(Qs, As, Qt, At):
    """Exchange that leaves source and target at the common averaged
    density U = (Qs + Qt)/(As + At): the source ends at As*U."""
    U = (np.asarray(Qs) + np.asarray(Qt)) / (As + At)
    return As * U - np.asarray(Qs)


# --------------------------------------------------------------------------
# mixing
# --------------------------------------------------------------------------
class MixCase:
    """Material 0 on a 5x5 grid (material 1 is inert: full where alpha^0 = 0,
    empty elsewhere, never a source)."""

    def __init__(self, nx=5, ny=5):
        self.nx, self.ny = nx, ny
        self.o = oracle.Oracle(cfg2(nx, ny))
        self.phi = np.ones((ny, nx))
        self.chi = np.ones((ny, nx), np.int32)
        self.al = np.zeros((2, ny, nx))
        self.Q = np.zeros((2, 4, ny, nx))

    def cell(self, i, j, chi, phi, alpha, Q=None):
        self.chi[j, i] = chi
        self.phi[j, i] = phi
        self.al[0, j, i] = alpha
        if Q is not None:
            self.Q[0, :, j, i] = Q

    def run(self, full=False):
        self.al[1] = np.where(self.al[0] > 0.0, 0.0, 1.0)
        self.al[1][self.chi == 1] = 1.0 - self.al[0][self.chi == 1]
        self.Q[1] = 0.0
        self.Q[1, 0] = self.al[1]  # a uniform state of material 1
        self.Q[1, 3] = 2.5 * self.al[1]
        d0 = self.o.diag()
        out = self.o.mix(self.Q, self.al, self.phi, self.chi)
        d1 = self.o.diag()
        self.absorbed = d1["n_absorb"] - d0["n_absorb"]
        if full:
            return out, d1["n_mixsrc"] - d0["n_mixsrc"], d1["n_stranded"] - d0["n_stranded"]
        # material 1 never mixes here
        assert np.array_equal(out[1], self.Q[1])
        return out[0], d1["n_mixsrc"] - d0["n_mixsrc"], d1["n_stranded"] - d0["n_stranded"]


def test_mixing_three_targets_weights_4_1_2():
    """Source (2,2) of material 0 (centre in material 1, alpha 1/4).  The
    level set gives g_x = 0.5, g_y = 0.25, so the x, y and diagonal targets
    (all full cells of material 0) weigh g_x^2 : g_y^2 : |g_x g_y| =
    4 : 1 : 2, i.e. beta = (4/7, 1/7, 2/7).  (|g| weights would give
    4 : 2 : 1; no diagonal, 4/5 and 1/5.)"""
    c = MixCase()
    Qs = np.array([0.25, 0.125, -0.0625, 0.5])
    Qx, Qy, Qd = (np.array([2.0, 1.0, 0.0, 5.0]), np.array([3.0, 0.0, 1.0, 6.0]),
                  np.array([4.0, -1.0, 0.5, 8.0]))
    c.cell(2, 2, 1, 0.5, 0.25, Qs)
    c.cell(3, 2, 0, 0.25, 1.0, Qx)   # lsv +0.25
    c.cell(1, 2, 1, 0.25, 0.0)       # lsv -0.25 -> g_x = 0.5
    c.cell(2, 3, 0, 0.125, 1.0, Qy)  # lsv +0.125
    c.cell(2, 1, 1, 0.125, 0.0)      # lsv -0.125 -> g_y = 0.25
    c.cell(3, 3, 0, 1.0, 1.0, Qd)
    out, nsrc, nstr = c.run()
    assert (nsrc, nstr) == (1, 0)
    beta = {(3, 2): 4.0 / 7.0, (2, 3): 1.0 / 7.0, (3, 3): 2.0 / 7.0}
    Qt = {(3, 2): Qx, (2, 3): Qy, (3, 3): Qd}
    total = np.zeros(4)
    for (i, j), b in beta.items():
        m = b * pair_exchange(Qs, 0.25, Qt[(i, j)], 1.0)
        assert close(out[:, j, i], Qt[(i, j)] - m), (i, j)
        total += m
    assert close(out[:, 2, 2], Qs + total)
    # every other cell is untouched
    mask = np.ones((5, 5), bool)
    for (i, j) in [(2, 2), (3, 2), (2, 3), (3, 3)]:
        mask[j, i] = False
    assert np.array_equal(out[:, mask], c.Q[0][:, mask])
    # conservation of every component
    assert close(out.sum(axis=(1, 2)), c.Q[0].sum(axis=(1, 2)))


def test_mixing_single_target_averages_the_pair():
    """One eligible target (the x neighbour; g_y = 0 so no y or diagonal
    target): source and target end with the same conserved density, the
    volume-weighted average (Q_s + Q_t)/(alpha_s + alpha_t)."""
    c = MixCase()
    Qs = np.array([0.3, -0.6, 0.15, 1.2])
    Qt = np.array([1.6, 0.4, -0.2, 4.0])
    c.cell(2, 2, 1, 0.5, 0.3, Qs)
    c.cell(1, 2, 0, 0.5, 0.8, Qt)   # lsv +0.5 (side of increasing phi^0)
    c.cell(3, 2, 1, 0.5, 0.0)       # lsv -0.5 -> g_x = -1.0
    c.cell(2, 1, 1, 0.7, 0.0)
    c.cell(2, 3, 1, 0.7, 0.0)       # g_y = 0
    out, nsrc, _ = c.run()
    assert nsrc == 1
    U = (Qs + Qt) / 1.1
    assert close(out[:, 2, 2], 0.3 * U)
    assert close(out[:, 2, 1], 0.8 * U)


def test_mixing_new_cell_takes_the_neighbours_density():
    """A new cell (alpha > 0, empty state) fills at the neighbour's averaged
    density: Q_s' = alpha_s Q_t/(alpha_s + alpha_t)."""
    c = MixCase()
    Qt = np.array([2.0, 1.0, 0.5, 6.0])
    c.cell(2, 2, 1, 0.5, 0.25, np.zeros(4))
    c.cell(3, 2, 0, 0.5, 1.0, Qt)
    c.cell(1, 2, 1, 0.5, 0.0)
    out, nsrc, _ = c.run()
    assert nsrc == 1
    assert close(out[:, 2, 2], 0.25 * Qt / 1.25)
    assert close(out[:, 2, 3], 1.0 * Qt / 1.25)


def test_mixing_own_partial_cell_without_mass_fills_like_a_new_cell():
    """A part of the cell's own material with alpha_mix <= alpha < 1 whose
    partial density is roundoff (here negative) is filled like a new cell:
    the pair ends at the averaged density (Q_s + Q_t)/(alpha_s + alpha_t).
    With positive mass, or with alpha = 1, the same cell is no source."""
    Qt = np.array([2.0, 1.0, 0.5, 6.0])
    junk = np.array([-1e-18, 3e-19, 0.0, 2e-17])

    def case(alpha, Qs):
        c = MixCase()
        c.cell(2, 2, 0, 0.5, alpha, Qs)  # the cell's own material
        c.cell(3, 2, 0, 0.5, 1.0, Qt)    # lsv +0.5: the target side
        c.cell(1, 2, 1, 0.5, 0.0)        # lsv -0.5 -> g_x = 1
        c.cell(2, 1, 1, 0.7, 0.0)
        c.cell(2, 3, 1, 0.7, 0.0)        # g_y = 0
        return c.run()

    out, nsrc, _ = case(0.6, junk)
    assert nsrc == 1
    U = (junk + Qt) / 1.6
    assert close(out[:, 2, 2], 0.6 * U)
    assert close(out[:, 2, 3], 1.0 * U)
    assert out[0, 2, 2] > 0.0
    Qm = np.array([0.9, 0.1, 0.0, 2.0])
    out, nsrc, _ = case(0.6, Qm)
    assert nsrc == 0 and np.array_equal(out[:, 2, 2], Qm)
    out, nsrc, _ = case(1.0, junk)
    assert nsrc == 0 and np.array_equal(out[:, 2, 2], junk)


def test_mixing_only_diagonal_target():
    """The x and y neighbours hold none of material 0 (ineligible, and not
    sources themselves); the diagonal neighbour is a full cell: it takes the
    whole exchange (beta = 1)."""
    c = MixCase()
    Qs = np.array([0.2, 0.1, 0.0, 0.7])
    Qd = np.array([0.9, 0.0, 0.45, 3.0])
    c.cell(2, 2, 1, 0.5, 0.2, Qs)
    c.cell(3, 2, 1, 0.1, 0.0)   # lsv -0.1
    c.cell(1, 2, 1, 0.3, 0.0)   # lsv -0.3 -> g_x = 0.2
    c.cell(2, 3, 1, 0.05, 0.0)  # lsv -0.05
    c.cell(2, 1, 1, 0.2, 0.0)   # lsv -0.2 -> g_y = 0.15
    c.cell(3, 3, 0, 0.5, 0.9, Qd)
    out, nsrc, nstr = c.run()
    assert (nsrc, nstr) == (1, 0)
    U = (Qs + Qd) / 1.1
    assert close(out[:, 2, 2], 0.2 * U)
    assert close(out[:, 3, 3], 0.9 * U)


def test_mixing_fallback_largest_neighbour_lowest_index():
    """No eligible x / y / diagonal target on the side of increasing phi^0:
    the 8-neighbour of largest alpha (>= alpha_mix, chi = 0) takes all; of
    two equal ones, the lower linear index (3,1) wins over (1,3); a smaller
    one (1,1) loses."""
    c = MixCase()
    Qs = np.array([0.1, 0.05, 0.0, 0.3])
    Qa, Qb, Qc = (np.array([0.8, 0.0, 0.0, 2.0]), np.array([1.6, 0.0, 0.0, 4.0]),
                  np.array([0.7, 0.0, 0.0, 1.0]))
    c.cell(2, 2, 1, 0.5, 0.1, Qs)
    c.cell(3, 2, 1, 0.2, 0.0)
    c.cell(1, 2, 1, 0.4, 0.0)   # g_x = 0.2 > 0
    c.cell(2, 3, 1, 0.2, 0.0)
    c.cell(2, 1, 1, 0.4, 0.0)   # g_y = 0.2 > 0; (3,3) holds none of material 0
    c.cell(3, 1, 0, 0.5, 0.8, Qa)
    c.cell(1, 3, 0, 0.5, 0.8, Qb)
    c.cell(1, 1, 0, 0.5, 0.7, Qc)
    out, nsrc, nstr = c.run()
    assert (nsrc, nstr) == (1, 0)
    U = (Qs + Qa) / 0.9
    assert close(out[:, 2, 2], 0.1 * U)
    assert close(out[:, 1, 3], 0.8 * U)
    assert np.array_equal(out[:, 3, 1], Qb)
    assert np.array_equal(out[:, 1, 1], Qc)


def test_mixing_stranded_source_joins_the_cells_material():
    """No neighbour of material 0 at all, in a cell of material 1: the
    source's conserved quantities are added to material 1's in the same cell
    (exactly), material 0 is left empty there, nothing else changes, and the
    source is counted as absorbed, not stranded."""
    c = MixCase()
    Qs = np.array([0.1, 0.05, 0.0, 0.3])
    c.cell(2, 2, 1, 0.5, 0.1, Qs)
    c.cell(3, 2, 1, 0.2, 0.0)
    c.cell(1, 2, 1, 0.4, 0.0)
    out, nsrc, nstr = c.run(full=True)
    assert (nsrc, nstr, c.absorbed) == (1, 0, 1)
    assert np.array_equal(out[0], np.zeros_like(out[0]))
    # material 1 of the cell: alpha 0.9 of (1, 0, 0, 2.5) plus Q_s
    assert np.array_equal(out[1, :, 2, 2], np.array([0.9 + 0.1, 0.05, 0.0, 2.25 + 0.3]))
    keep = np.ones((c.ny, c.nx), bool)
    keep[2, 2] = False
    assert np.array_equal(out[1][:, keep], c.Q[1][:, keep])


def test_mixing_stranded_own_material_goes_to_largest_other():
    """Three materials; cell (2,2) belongs to material 0, which fills only
    0.3 of it, with no other cell of material 0 around (a fragment): its
    state joins material 2 (alpha 0.45), not material 1 (alpha 0.25), in the
    cell, and the cell is counted as relabelled (the indicator itself changes
    in the step, see test_stranded_fragment_is_relabelled_in_a_step)."""
    nx = ny = 5
    o = oracle.Oracle(cfg2(nx, ny, M=3))
    phi = np.ones((ny, nx))
    chi = np.ones((ny, nx), np.int32)
    al = np.zeros((3, ny, nx))
    al[1] = 1.0
    al[:, 2, 2] = (0.3, 0.25, 0.45)
    chi[2, 2] = 0
    phi[2, 2] = 0.05
    Q = np.zeros((3, 4, ny, nx))
    for m in range(3):
        Q[m, 0] = al[m] * (1.0 + m)
        Q[m, 3] = al[m] * (2.0 + m)
    d0 = o.diag()
    out = o.mix(Q, al, phi, chi)
    d1 = o.diag()
    assert d1["n_relabel"] - d0["n_relabel"] == 1
    assert d1["n_absorb"] - d0["n_absorb"] == 1
    assert np.array_equal(out[0, :, 2, 2], np.zeros(4))
    assert np.array_equal(out[2, :, 2, 2], Q[2, :, 2, 2] + Q[0, :, 2, 2])
    assert np.array_equal(out[1], Q[1])


def test_mixing_vanishing_source_hands_over_exactly():
    """A vanishing cell (alpha = 0, state left over) with three targets of
    equal weight (g_x = g_y, full cells): each of the first two receives
    Q_s/3, the last the exact remainder, so the source ends at exactly 0 and
    the total is unchanged bit for bit."""
    c = MixCase()
    Qs = np.array([0.1, 0.3, 0.7, 1.1])
    T = {(3, 2): np.array([1.0, 0.0, 0.0, 2.5]), (2, 3): np.array([2.0, 0.0, 0.0, 5.0]),
         (3, 3): np.array([3.0, 0.0, 0.0, 7.5])}
    c.cell(2, 2, 1, 0.5, 0.0, Qs)
    c.cell(1, 2, 1, 0.5, 0.0)
    c.cell(2, 1, 1, 0.5, 0.0)
    for (i, j), q in T.items():
        c.cell(i, j, 0, 0.5, 1.0, q)
    out, nsrc, _ = c.run()
    assert nsrc == 1
    assert np.array_equal(out[:, 2, 2], np.zeros(4))
    third = Qs * (1.0 / 3.0)
    assert close(out[:, 2, 3], T[(3, 2)] + third)
    assert close(out[:, 3, 2], T[(2, 3)] + third)
    assert close(out[:, 3, 3], T[(3, 3)] + (Qs - third - third))
    # the received amounts add up to the source's state exactly
    got = (out[:, 2, 3] - T[(3, 2)], out[:, 3, 2] - T[(2, 3)], out[:, 3, 3] - T[(3, 3)])
    # without the exact remainder three thirds would not cancel Q_s here
    naive = ((Qs - third) - third) - third
    assert np.any(naive != 0.0)
    assert close(got[0] + got[1] + got[2], Qs, 1e-15)


def test_mixing_1d_source_and_face_aligned_vanishing_cell():
    """1D (x targets only, beta = 1).  Cell 5 of material 0 (centre in
    material 1, alpha 0.4) mixes with cell 4; cell 8 (alpha 0: the
    interface lies on its face) still holds state of material 0 and hands it
    all to cell 7."""
    o = oracle.Oracle(cfg1(12))
    phi = np.abs(np.arange(12) - 4.6) + 0.0
    chi = np.where(np.arange(12) <= 4, 0, 1).astype(np.int32)
    chi[7] = 0
    phi[7] = 0.5
    phi[8] = 0.5
    phi[6] = 0.5
    al = np.zeros((2, 12))
    al[0, :5] = 1.0
    al[0, 5] = 0.4
    al[0, 7] = 1.0
    al[1] = 1.0 - al[0]
    Q = np.zeros((2, 3, 12))
    Q[0, 0, :5] = 1.0
    Q[0, 2, :5] = 2.5
    Q[0, :, 5] = [0.2, 0.1, 0.6]
    Q[0, :, 7] = [1.5, 0.0, 3.0]
    Q[0, :, 8] = [0.01, 0.002, 0.03]
    Q[1, 0] = al[1] * 0.5
    Q[1, 2] = al[1] * 1.0
    out = o.mix(Q, al, phi, chi)
    U = (Q[0, :, 5] + Q[0, :, 4]) / 1.4
    out = out[:, :, 0, :]
    assert close(out[0, :, 5], 0.4 * U)
    assert close(out[0, :, 4], 1.0 * U)
    assert np.array_equal(out[0, :, 8], np.zeros(3))
    assert close(out[0, :, 7], Q[0, :, 7] + Q[0, :, 8])
    assert close(out[0].sum(axis=-1), Q[0].sum(axis=-1))
    assert np.array_equal(out[1], Q[1])


# --------------------------------------------------------------------------
# ghost-state extension
# --------------------------------------------------------------------------
def test_extension_1d_constant_from_the_interface_cell():
    """Material 0 real in cells 0..4 (distinct states), material 1 real in
    5..11; the interface lies on the face 4|5.  Upwind sweeps along
    increasing phi^0 give cells 5..8 (the 4-cell band) exactly W^0_4, and
    cells 1..4 exactly W^1_5; farther cells stay empty."""
    n = 12
    o = oracle.Oracle(cfg1(n))
    x = np.arange(n)
    phi = np.abs(x - 4.5)
    chi = np.where(x <= 4, 0, 1).astype(np.int32)
    W = np.zeros((2, 4, 1, n))
    valid = np.zeros((2, 1, n), np.uint8)
    for i in range(5):
        W[0, :, 0, i] = [1.0 + i, 0.1 * i, 0.0, 2.0 + i]
        valid[0, 0, i] = 1
    for i in range(5, n):
        W[1, :, 0, i] = [0.5 + 0.1 * i, -0.2, 0.0, 1.0 + i]
        valid[1, 0, i] = 1
    Wo, vo = o.extend(phi, chi, W, valid)
    for i in range(5, 9):
        assert vo[0, 0, i] == 1
        assert np.array_equal(Wo[0, :, 0, i], W[0, :, 0, 4]), i
    assert vo[0, 0, 9:].sum() == 0
    for i in range(1, 5):
        assert vo[1, 0, i] == 1
        assert np.array_equal(Wo[1, :, 0, i], W[1, :, 0, 5]), i
    assert vo[1, 0, 0] == 0
    # real states are untouched
    assert np.array_equal(Wo[0, :, 0, :5], W[0, :, 0, :5])


def test_extension_2d_weights_are_the_gradient_components():
    """Material 0 real in the L-shaped region i <= 1 or j <= 1 of a 6x6 grid.
    At the ghost cell (2,2) the level set gives g_x = -2, g_y = -1, both
    upwind neighbours (1,2) and (2,1) are real: W = (2 W_(1,2) + W_(2,1))/3.
    At (2,3) only g_x is non-zero: W = W_(1,3).  (Squared weights would give
    (4 W_(1,2) + W_(2,1))/5; a flipped upwind side would take no value.)"""
    o = oracle.Oracle(cfg2(6, 6, k_ext=8))
    chi = np.ones((6, 6), np.int32)
    valid = np.zeros((2, 6, 6), np.uint8)
    W = np.zeros((2, 4, 6, 6))
    for j in range(6):
        for i in range(6):
            if i <= 1 or j <= 1:
                chi[j, i] = 0
                valid[0, j, i] = 1
                W[0, :, j, i] = [1.0 + i + 2 * j, 0.1 * i, 0.2 * j, 5.0 + j]
            else:
                valid[1, j, i] = 1
                W[1, :, j, i] = [0.5, 0.0, 0.0, 1.0]
    W[0, :, 2, 1] = [3.0, 0.3, 0.6, 9.0]
    W[0, :, 1, 2] = [6.0, 0.9, 0.3, 3.0]
    phi = np.ones((6, 6))
    phi[2, 3] = phi[2, 1] = 1.0   # g_x(2,2) = -1 - 1 = -2
    phi[3, 2] = phi[1, 2] = 0.5   # g_y(2,2) = -0.5 - 0.5 = -1
    phi[3, 3] = 1.0
    phi[3, 1] = 1.0
    phi[4, 2] = 0.5               # g_y(2,3) = -0.5 - (-0.5) = 0
    Wo, vo = o.extend(phi, chi, W, valid)
    assert vo[0, 2, 2] == 1
    assert close(Wo[0, :, 2, 2], [4.0, 0.5, 0.5, 7.0])
    assert np.array_equal(Wo[0, :, 3, 2], W[0, :, 3, 1])


def test_extension_mean_sweeps_are_jacobi_over_valid_neighbours():
    """With no upwind sweeps (k_ext = 0) and a flat level set, two real cells
    a = (0,0) and b = (2,0) fill the rest by 4 sweeps of the mean of the
    valid 8-neighbours, each sweep from the previous one's values:
    sweep 1: (1,0) = (1,1) = (a+b)/2, (0,1) = a, (2,1) = b, (3,0) = (3,1) = b;
    sweep 2: (0,2) = (a + (a+b)/2)/2 = (3a+b)/4."""
    o = oracle.Oracle(cfg2(5, 5, k_ext=0))
    chi = np.ones((5, 5), np.int32)
    chi[0, 0] = chi[0, 2] = 0
    valid = np.zeros((2, 5, 5), np.uint8)
    W = np.zeros((2, 4, 5, 5))
    a = np.array([1.0, 0.5, -0.25, 2.0])
    b = np.array([3.0, -0.5, 0.75, 6.0])
    W[0, :, 0, 0], W[0, :, 0, 2] = a, b
    valid[0, 0, 0] = valid[0, 0, 2] = 1
    phi = np.ones((5, 5))
    Wo, vo = o.extend(phi, chi, W, valid)
    assert vo[0].all()
    assert close(Wo[0, :, 0, 1], (a + b) / 2)
    assert close(Wo[0, :, 1, 1], (a + b) / 2)
    assert close(Wo[0, :, 1, 0], a)
    assert close(Wo[0, :, 1, 2], b)
    assert close(Wo[0, :, 0, 3], b)
    assert close(Wo[0, :, 1, 3], b)
    assert close(Wo[0, :, 2, 0], (3 * a + b) / 4)


# --------------------------------------------------------------------------
# level-set velocity
# --------------------------------------------------------------------------
def test_ls_velocity_1d_carried_four_cells():
    """The interface cell 5 has S_M = 0.7.  With phi = |i - 5| (inside the
    band of 8 cells) the sweeps towards smaller phi carry 0.7 to cells 1..9;
    cells 0 and 10, 11 keep their material's velocity (0.2 where a state is
    valid) or 0 (none)."""
    n = 12
    o = oracle.Oracle(cfg1(n))
    x = np.arange(n)
    phi = np.abs(x - 5.0)
    chi = np.where(x <= 5, 0, 1).astype(np.int32)
    v = np.zeros((2, 1, n))
    v[0, 0, 5] = 0.7
    vok = np.zeros((1, n), np.uint8)
    vok[0, 5] = 1
    W = np.zeros((2, 4, 1, n))
    valid = np.zeros((2, 1, n), np.uint8)
    W[1, 1, 0, 10] = 0.2
    W[1, 1, 0, 11] = 0.2
    valid[1, 0, 10] = valid[1, 0, 11] = 1
    out = o.ls_velocity(phi, chi, v, vok, W, valid)
    expect = np.zeros(n)
    expect[1:10] = 0.7
    expect[10:] = 0.2
    assert np.array_equal(out[0, 0], expect)


def test_ls_velocity_2d_weights_are_the_gradient_components():
    """Interface cells (1,2) with v = (1, 0) and (2,1) with v = (0, 1); at
    (2,2) phi rises by 2 in x and 1 in y across the cell: v = (2 (1,0) +
    1 (0,1))/3 = (2/3, 1/3)."""
    o = oracle.Oracle(cfg2(5, 5))
    phi = np.full((5, 5), 3.0)
    phi[2, 1], phi[2, 3] = 0.0, 2.0    # g_x = 2
    phi[1, 2], phi[3, 2] = 0.5, 1.5    # g_y = 1
    phi[2, 2] = 1.0
    chi = np.zeros((5, 5), np.int32)
    v = np.zeros((2, 5, 5))
    vok = np.zeros((5, 5), np.uint8)
    v[:, 2, 1] = [1.0, 0.0]
    v[:, 1, 2] = [0.0, 1.0]
    vok[2, 1] = vok[1, 2] = 1
    W = np.zeros((2, 4, 5, 5))
    valid = np.zeros((2, 5, 5), np.uint8)
    out = o.ls_velocity(phi, chi, v, vok, W, valid)
    assert close(out[:, 2, 2], [2.0 / 3.0, 1.0 / 3.0])
    # set cells keep their value
    assert np.array_equal(out[:, 2, 1], [1.0, 0.0])
