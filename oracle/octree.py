"""FP64 oracle of the Barnes-Hut octree force in the S1 x R2 topology.

TEST INFRASTRUCTURE (see the package docstring).

The paper's octree (Sect. 2.4, "Octree"): cubic cells, a root cell twice the
largest linear size of the volume (the cylinder's height or diameter),
random shifts of the domain along the axis and rotations about it at every
step, and a radial correction table measured on the initial load with the
same tree parameters and subtracted from the tree forces.  What the paper
leaves open is fixed here (each is a reading):

* Frame.  Positions are rotated by ``angle`` about the axis and shifted by
  ``shift`` along it (z wrapped into [0, L)); the root cube has side
  S0 = 2 max(L, 2 R_dom) and centre (0, 0, L/2).  Accelerations are rotated
  back at the end.
* Cells.  Integer cell coordinates q = floor((p - lo) 2^21 / S0), clamped to
  [0, 2^21 - 1], interleaved into a 63-bit Morton key (x bit above y bit
  above z bit per level).  A cell is split into its octants when it holds
  more than ``leaf_size`` particles and is above level 21.  The cells form
  a list in depth-first order (children by octant) with, for each cell, the
  index of the first cell after its subtree ("skip").
* Multipoles.  A cell acts through its mass at its centre of mass and,
  optionally, its traceless quadrupole about the centre of mass,
  Q_ab = sum m (3 y_a y_b - |y|^2 delta_ab), y = x - x_com, which adds
  Q s / r^5 - (5/2) (s.Q.s) s / r^7 to the acceleration at separation s
  (target minus centre of mass) for each image |n| <= 4 about the minimum
  image (the table's band beyond carries only the monopole: the quadrupole
  term falls as 1/n^4).
* Groups.  Targets walk the tree in groups of at most ``group`` particles
  made of whole sibling cells: for every cell holding more than ``group``
  particles, its children (in order) that hold at most ``group`` are packed
  greedily into runs of at most ``group`` particles (a leaf holding more is
  cut into consecutive runs); a tree with at most ``group`` particles is one
  group.  A group accepts a cell when (S0/2^level)^2 < theta^2 d^2 and
  d^2 > (h_group + h_cell)^2 (compared squared, as written), with d the
  periodic (minimum over the images z_c, z_c +- L) distance from the cell's
  centre of mass to the group's bounding box, h_group and h_cell the largest
  softening lengths.  Group size 1 is
  the classical per-particle criterion.  An accepted cell adds its monopole
  to every target of the group, an opened leaf its particles (self pairs
  skipped).
* Interactions.  Both are the pair interaction of the tabulated scheme:
  the images |n| <= 1 (spline-softened; beyond the softening for cells)
  plus the band from a correction table (``oracle.table``).  With theta = 0
  no cell is ever accepted and the tree force is the direct tabulated force.
* Radial correction.  The mean radial error (tree minus direct) of the load
  in ``n_bins`` equal bins of rho on [0, R_dom], accumulated over the given
  (shift, angle) realisations; applied by linear interpolation between bin
  centres (constant beyond the first and last centre).
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from oracle import table as ot

KEY_LEVELS = 21


def transform(pos, L, shift, angle):
    c, s = math.cos(angle), math.sin(angle)
    x = c * pos[0] - s * pos[1]
    y = s * pos[0] + c * pos[1]
    z = pos[2] + shift
    z = z - L * np.floor(z / L)
    z = np.where(z >= L, 0.0, z)
    return np.stack([x, y, z])


def root_cube(L, R_dom):
    side = 2.0 * max(L, 2.0 * R_dom)
    lo = np.array([-0.5 * side, -0.5 * side, 0.5 * L - 0.5 * side])
    return lo, side


def morton_keys(pos_t, lo, side):
    scale = float(1 << KEY_LEVELS) / side
    q = np.floor((pos_t - lo[:, None]) * scale)
    q = np.clip(q, 0, (1 << KEY_LEVELS) - 1).astype(np.int64)
    key = np.zeros(pos_t.shape[1], dtype=np.int64)
    for b in range(KEY_LEVELS):
        key |= ((q[0] >> b) & 1) << (3 * b + 2)
        key |= ((q[1] >> b) & 1) << (3 * b + 1)
        key |= ((q[2] >> b) & 1) << (3 * b)
    return key


class Tree:
    """Cells in depth-first order: level, [start, end) in key order, mass,
    centre of mass (3), largest softening, leaf flag, skip index."""

    def __init__(self, pos, mass, eps, L, R_dom, shift=0.0, angle=0.0, leaf_size=16, quadrupole=False):
        self.L, self.leaf_size = float(L), int(leaf_size)
        self.lo, self.side = root_cube(L, R_dom)
        self.pos_t = transform(np.asarray(pos, dtype=np.float64), L, shift, angle)
        self.keys = morton_keys(self.pos_t, self.lo, self.side)
        N = self.keys.size
        self.order = np.lexsort((np.arange(N), self.keys))   # key, then index
        self.skey = self.keys[self.order]
        self.sp = self.pos_t[:, self.order]
        self.sm = np.asarray(mass, dtype=np.float64)[self.order]
        self.sh = np.asarray(eps, dtype=np.float64)[self.order]
        self.cells = []
        self._build(0, 0, N)
        self.level = np.array([c[0] for c in self.cells])
        self.start = np.array([c[1] for c in self.cells])
        self.end = np.array([c[2] for c in self.cells])
        self.mass = np.array([c[3] for c in self.cells])
        self.com = np.array([c[4] for c in self.cells]).T
        self.hmax = np.array([c[5] for c in self.cells])
        self.leaf = np.array([c[6] for c in self.cells])
        self.skip = np.array([c[7] for c in self.cells])
        self.quad = np.zeros((6, len(self.cells)))   # xx, yy, zz, xy, xz, yz
        if quadrupole:
            for k in range(len(self.cells)):
                sl = slice(self.start[k], self.end[k])
                y = self.sp[:, sl] - self.com[:, k:k + 1]
                m = self.sm[sl]
                y2 = (y * y).sum(axis=0)
                self.quad[:, k] = [np.sum(m * (3 * y[0] * y[0] - y2)), np.sum(m * (3 * y[1] * y[1] - y2)),
                                   np.sum(m * (3 * y[2] * y[2] - y2)), np.sum(m * 3 * y[0] * y[1]),
                                   np.sum(m * 3 * y[0] * y[2]), np.sum(m * 3 * y[1] * y[2])]

    def _build(self, level, start, end):
        m = self.sm[start:end]
        M = m.sum()
        if M > 0:
            com = (self.sp[:, start:end] * m).sum(axis=1) / M
        else:  # massless cell: its geometric centre
            q = self.skey[start]
            com = self.lo + (self._cell_corner(q, level) + 0.5) * (self.side / (1 << level))
        leaf = (end - start) <= self.leaf_size or level == KEY_LEVELS
        idx = len(self.cells)
        self.cells.append([level, start, end, M, com, self.sh[start:end].max(), leaf, -1])
        if not leaf:
            shift = 3 * (KEY_LEVELS - level - 1)
            digit = (self.skey[start:end] >> shift) & 7
            s = start
            for oc in range(8):
                e = s + int(np.count_nonzero(digit == oc))
                if e > s:
                    self._build(level + 1, s, e)
                s = e
        self.cells[idx][7] = len(self.cells)

    @staticmethod
    def _cell_corner(key, level):
        q = np.zeros(3)
        for b in range(level):
            digit = (int(key) >> (3 * (KEY_LEVELS - 1 - b))) & 7
            q = 2 * q + np.array([(digit >> 2) & 1, (digit >> 1) & 1, digit & 1])
        return q

    def size(self, k):
        return self.side / (1 << int(self.level[k]))


def groups(T, G):
    """Target groups as (start, count) ranges in key order (see above)."""
    cnt = T.end - T.start
    if cnt[0] <= G:
        return [(0, int(cnt[0]))]
    out = []
    for c in range(len(T.cells)):
        if cnt[c] <= G:
            continue
        if T.leaf[c]:
            out += [(s, min(G, T.end[c] - s)) for s in range(T.start[c], T.end[c], G)]
            continue
        run_s, run_n = 0, 0
        ch = c + 1
        while ch < T.skip[c]:
            if cnt[ch] > G:
                if run_n:
                    out.append((run_s, run_n))
                run_n = 0
            else:
                if run_n + cnt[ch] > G:
                    out.append((run_s, run_n))
                    run_n = 0
                if run_n == 0:
                    run_s = int(T.start[ch])
                run_n += int(cnt[ch])
            ch = T.skip[ch]
        if run_n:
            out.append((run_s, run_n))
    return out


def box_distance2(c, lo, hi, L):
    """Squared distance from point c to the box [lo, hi], periodic along z."""
    dx = max(0.0, lo[0] - c[0], c[0] - hi[0])
    dy = max(0.0, lo[1] - c[1], c[1] - hi[1])
    dz = min(max(0.0, lo[2] - cz, cz - hi[2]) for cz in (c[2] - L, c[2], c[2] + L))
    return dx * dx + dy * dy + dz * dz


QUAD_IMAGES = 4


def _quadrupole(tree, tg, c, q, acc):
    """Quadrupole term of one cell (centre of mass c, moments q) on the
    targets tg, images |n| <= QUAD_IMAGES about the minimum image."""
    L = tree.L
    tp = tree.sp[:, tg]
    t = tp[2] - c[2]
    d = t - L * np.floor(t / L + 0.5)
    Q = np.array([[q[0], q[3], q[4]], [q[3], q[1], q[5]], [q[4], q[5], q[2]]])
    for n in range(-QUAD_IMAGES, QUAD_IMAGES + 1):
        s = np.stack([tp[0] - c[0], tp[1] - c[1], d - n * L])
        r2 = (s * s).sum(axis=0)
        Qs = Q @ s
        sQs = (s * Qs).sum(axis=0)
        acc[:, tg] += Qs / r2 ** 2.5 - 2.5 * sQs * s / r2 ** 3.5


def _interact(tree, tg, src_pos, src_m, src_h, src_id, tab, order, acc):
    """Targets tg (sorted indices) against sources: near images + band."""
    L = tree.L
    tp = tree.sp[:, tg]
    acc[:, tg] += oracle.pairs(tp, tree.sh[tg], tg, src_pos, src_m, src_h, src_id, L, 1)
    keep = src_id[None, :] != tg[:, None]                      # (T, S)
    dx = (tp[0][:, None] - src_pos[0][None, :])[keep]
    dy = (tp[1][:, None] - src_pos[1][None, :])[keep]
    t = (tp[2][:, None] - src_pos[2][None, :])[keep]
    d = t - L * np.floor(t / L + 0.5)
    m = np.broadcast_to(src_m[None, :], keep.shape)[keep]
    row = np.broadcast_to(np.arange(tg.size)[:, None], keep.shape)[keep]
    bx, by, bz = ot.band_pairs(dx, dy, d, L, tab, order)
    for c, b in enumerate((bx, by, bz)):
        acc[c, tg] += np.bincount(row, weights=m * b, minlength=tg.size)


def tree_forces(pos, mass, eps, L, R_dom, tab, order, theta, shift=0.0, angle=0.0,
                leaf_size=16, group=64, stats=None, targets=None, quadrupole=False):
    """Accelerations (3, N) of every particle by the octree (G = 1), in the
    original frame and order; with ``targets`` (original indices) only the
    groups holding them are walked and (3, len(targets)) is returned."""
    T = Tree(pos, mass, eps, L, R_dom, shift, angle, leaf_size, quadrupole)
    N = T.sm.size
    acc = np.zeros((3, N))     # in key order, transformed frame
    n_cell = n_part = 0
    gl = sorted(groups(T, group))             # by start (cells emit them in depth-first order)
    if targets is not None:
        where = np.empty(N, dtype=np.int64)
        where[T.order] = np.arange(N)            # key-order position of each particle
        starts = np.array([g[0] for g in gl])
        keep = np.unique(np.searchsorted(starts, where[np.asarray(targets)], side="right") - 1)
        gl = [gl[k] for k in keep]
    for g0, gn in gl:
        tg = np.arange(g0, g0 + gn)
        lo = T.sp[:, tg].min(axis=1)
        hi = T.sp[:, tg].max(axis=1)
        hg = T.sh[tg].max()
        k = 0
        theta2 = theta * theta
        while k < len(T.cells):
            d2 = box_distance2(T.com[:, k], lo, hi, L)
            hs = hg + T.hmax[k]
            if T.size(k) * T.size(k) < theta2 * d2 and d2 > hs * hs:
                _interact(T, tg, T.com[:, k:k + 1], T.mass[k:k + 1], T.hmax[k:k + 1],
                          np.array([-1]), tab, order, acc)
                if quadrupole:
                    _quadrupole(T, tg, T.com[:, k], T.quad[:, k], acc)
                n_cell += tg.size
                k = T.skip[k]
            elif T.leaf[k]:
                s = np.arange(T.start[k], T.end[k])
                _interact(T, tg, T.sp[:, s], T.sm[s], T.sh[s], s, tab, order, acc)
                n_part += tg.size * s.size
                k = T.skip[k]
            else:
                k += 1
    if stats is not None:
        stats.update(cell_interactions=n_cell, particle_interactions=n_part, cells=len(T.cells))
    out = np.empty_like(acc)
    out[:, T.order] = acc
    c, s = math.cos(angle), math.sin(angle)
    ax = c * out[0] + s * out[1]
    ay = -s * out[0] + c * out[1]
    res = np.stack([ax, ay, out[2]])
    return res if targets is None else res[:, np.asarray(targets)]


# ---------------------------------------------------------------- radial correction
def radial_bins(pos, acc_err, R_dom, n_bins):
    """Per-bin sums and counts of the radial component of ``acc_err``."""
    rho = np.hypot(pos[0], pos[1])
    with np.errstate(invalid="ignore", divide="ignore"):
        fr = np.where(rho > 0, (acc_err[0] * pos[0] + acc_err[1] * pos[1]) / rho, 0.0)
    b = np.clip(np.floor(rho / R_dom * n_bins).astype(np.int64), 0, n_bins - 1)
    sums = np.bincount(b, weights=fr, minlength=n_bins)
    counts = np.bincount(b, minlength=n_bins).astype(np.float64)
    return sums, counts


def calibrate(pos, mass, eps, L, R_dom, tab, order, theta, shifts, angles, n_bins,
              leaf_size=16, group=64, quadrupole=False):
    """Mean radial error (tree - direct) per radial bin over the realisations."""
    direct = ot.forces_table(pos, mass, eps, L, tab, order)
    sums = np.zeros(n_bins)
    counts = np.zeros(n_bins)
    for s, a in zip(shifts, angles):
        t = tree_forces(pos, mass, eps, L, R_dom, tab, order, theta, s, a, leaf_size, group,
                        quadrupole=quadrupole)
        ds, dc = radial_bins(pos, t - direct, R_dom, n_bins)
        sums += ds
        counts += dc
    return np.where(counts > 0, sums / np.maximum(counts, 1.0), 0.0)


def apply_correction(pos, acc, corr, R_dom):
    """Subtract the interpolated radial error along rho-hat."""
    n = len(corr)
    rho = np.hypot(pos[0], pos[1])
    centres = (np.arange(n) + 0.5) * (R_dom / n)
    delta = np.interp(rho, centres, corr)
    out = acc.copy()
    with np.errstate(invalid="ignore", divide="ignore"):
        ux = np.where(rho > 0, pos[0] / rho, 0.0)
        uy = np.where(rho > 0, pos[1] / rho, 0.0)
    out[0] -= delta * ux
    out[1] -= delta * uy
    return out
