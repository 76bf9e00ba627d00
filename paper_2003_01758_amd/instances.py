"""Seeded synthetic polynomial programs shaped like the paper's workloads.

This module is the only source of random numbers in the project.  It builds
problem (P) of Sec. II-B -- minimise p subject to g_i <= 0 and h_j = 0 on a
box D -- as monomial coefficient tensors.  It holds no Bernstein arithmetic:
polynomial products, shifts and point evaluations use numpy.polynomial, and
the solvers (the CPU oracle and the HIP library) take its arrays as input.

Coefficient layout: a polynomial of multi-degree (n_1..n_l) is a C-ordered
array of shape (n_1+1, ..., n_l+1); entry [j_1, ..., j_l] multiplies
x_1^j_1 ... x_l^j_l (x_l varies fastest in memory).

Workloads (seed of instance k of workload c: PCG64(1_000_003*c + k)):
  0  "small":   l=2, D=[-1,1]^2, cost (4,4) N(0,1); 16 planted inequalities
                (4,4) with coefficients N(0,1)*2^-(a+b).
  1  "rtd":     l=2, goal-distance cost (6,6); 500 obstacle constraints (10,10)
                from one shifted template, planted feasible.
  2  "4d":      l=4, cost (4,4,4,4); 100 planted inequalities (4,4,4,4);
                2 planted equalities (2,2,2,2); coefficients N(0,1)*2^-|J|.
  3  "batch":   l in {2,3}, constraint degree in {4,6,8,10}, constraint count
                log-uniform in [50,1000], otherwise as workload 1.
  4  "serve":   l=2, workload-1 shapes, constraint count log-uniform in
                [100,2000].
  5  "waypoints": l=2, the multi-waypoint product cost (12,12); 100 obstacle
                constraints (10,10) as in workload 1.
  6  "rtdpop":  a planning problem built the way RTD builds it (Sec. II-C and
                Sec. VI): plans q = (speed, yaw rate) in Q = [0,1] x [-1,1];
                2 to 10 box obstacles of 30 cm ahead of the robot, seen as
                lidar points x_i on their outlines (48 to 240 points); one
                constraint w(x_i, q) + eps_q <= 0 per point, eps_q = 1e-4, from
                a synthetic FRS-like polynomial w (see frs_polynomial); the
                cost is the product over two waypoints of the squared distance
                of the plan's endpoint from each.  Nothing is planted: some
                plans are infeasible.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from numpy.polynomial import polynomial as npp

SEED_STRIDE = 1_000_003


@dataclasses.dataclass
class Instance:
    """One polynomial program (P) on a box, plus solver tolerances."""

    name: str
    l: int
    lo: np.ndarray            # (l,) float64
    hi: np.ndarray            # (l,) float64
    cost: np.ndarray          # l-dim coefficient tensor
    ineq: list                # list of l-dim coefficient tensors
    eq: list                  # list of l-dim coefficient tensors
    eps: float = 1e-3         # optimality tolerance (absolute, cost units)
    delta: float = 1e-4       # step tolerance (max box width, original coords)
    eps_eq: float = 1e-4      # equality tolerance
    max_boxes: int = 1 << 16  # M
    max_iters: int = 28       # N
    q0: np.ndarray | None = None   # planted feasible point (None if unknown)

    # ---- flat views in the C-ABI layout -------------------------------------------
    @property
    def cost_deg(self) -> np.ndarray:
        return np.array([s - 1 for s in self.cost.shape], dtype=np.int32)

    @property
    def n_ineq(self) -> int:
        return len(self.ineq)

    @property
    def n_eq(self) -> int:
        return len(self.eq)

    def _degs(self, polys) -> np.ndarray:
        if not polys:
            return np.zeros((0, self.l), dtype=np.int32)
        return np.array([[s - 1 for s in p.shape] for p in polys], dtype=np.int32)

    @property
    def ineq_deg(self) -> np.ndarray:
        return self._degs(self.ineq)

    @property
    def eq_deg(self) -> np.ndarray:
        return self._degs(self.eq)

    @staticmethod
    def _cat(polys) -> np.ndarray:
        if not polys:
            return np.zeros(0, dtype=np.float64)
        return np.concatenate([np.ascontiguousarray(p, dtype=np.float64).ravel()
                               for p in polys])

    @property
    def cost_flat(self) -> np.ndarray:
        return np.ascontiguousarray(self.cost, dtype=np.float64).ravel()

    @property
    def ineq_flat(self) -> np.ndarray:
        return self._cat(self.ineq)

    @property
    def eq_flat(self) -> np.ndarray:
        return self._cat(self.eq)

    def words_per_item(self) -> int:
        """Memory per item in words, 2l + Pi(P+1) + alpha*Pi(G+1) + beta*Pi(H+1)
        (Sec. IV-C, memory per item), with G and H the componentwise max degrees."""
        def common(polys):
            if not polys:
                return 0, 0
            g = np.max(self._degs(polys), axis=0) + 1
            return len(polys), int(np.prod(g))
        a, sg = common(self.ineq)
        b, sh = common(self.eq)
        return 2 * self.l + int(np.prod(self.cost.shape)) + a * sg + b * sh

    def with_options(self, **kw) -> "Instance":
        return dataclasses.replace(self, **kw)


# ---- polynomial helpers (numpy.polynomial; no Bernstein arithmetic) -------------------

def poly_eval(coef: np.ndarray, x) -> float:
    """Value of the tensor-coefficient polynomial at the point x (nested Horner
    through numpy.polynomial.polyval, last variable innermost)."""
    c = np.asarray(coef, dtype=np.float64)
    for k in range(c.ndim - 1, -1, -1):
        c = npp.polyval(float(x[k]), np.moveaxis(c, -1, 0))
    return float(c)


def poly_eval_many(coef: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Values at many points, pts of shape (n, l), via per-axis Vandermonde matrices."""
    c = np.asarray(coef, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, c.ndim)
    vs = [npp.polyvander(pts[:, k], c.shape[k] - 1) for k in range(c.ndim)]
    res = np.einsum("...j,nj->n...", c, vs[-1])
    for k in range(c.ndim - 2, -1, -1):
        res = np.einsum("n...j,nj->n...", res, vs[k])
    return res


def poly_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product of two tensor-coefficient polynomials (full N-d convolution)."""
    shape = tuple(sa + sb - 1 for sa, sb in zip(a.shape, b.shape))
    out = np.zeros(shape)
    for idx in np.ndindex(*a.shape):
        ca = a[idx]
        if ca == 0.0:
            continue
        sl = tuple(slice(i, i + sb) for i, sb in zip(idx, b.shape))
        out[sl] += ca * b
    return out


def poly_shift(coef: np.ndarray, s) -> np.ndarray:
    """Coefficients of q -> T(q - s) (per-axis composition with numpy.polynomial)."""
    c = np.asarray(coef, dtype=np.float64)
    for k in range(c.ndim):
        n = c.shape[k]
        # column j holds the coefficients of (q_k - s_k)^j
        basis = np.zeros((n, n))
        for j in range(n):
            basis[: j + 1, j] = npp.polypow([-float(s[k]), 1.0], j)
        c = np.moveaxis(np.tensordot(basis, np.moveaxis(c, k, 0), axes=(1, 0)), 0, k)
    return c


def _scaled_normal(rng, shape, base: float) -> np.ndarray:
    """N(0,1) coefficients scaled by base^-(total degree of the monomial)."""
    tot = np.zeros(shape)
    for k, s in enumerate(shape):
        sh = [1] * len(shape)
        sh[k] = s
        tot = tot + np.arange(s).reshape(sh)
    return rng.standard_normal(shape) * base ** (-tot)


def _planted(rng, p: np.ndarray, q0) -> np.ndarray:
    """g = p - p(q0) - U(0.1, 0.5): the planted point q0 is strictly feasible."""
    g = p.copy()
    g[(0,) * g.ndim] -= poly_eval(p, q0) + rng.uniform(0.1, 0.5)
    return g


def _goal_cost(rng, l: int, half_deg: int) -> np.ndarray:
    """Squared distance of a polynomial endpoint map e(q) from a seeded goal;
    each of the two components of e has multi-degree (half_deg,)*l, so the
    cost has multi-degree (2*half_deg,)*l."""
    shape = (half_deg + 1,) * l
    goal = rng.uniform(-2.0, 2.0, size=2)
    cost = np.zeros((2 * half_deg + 1,) * l)
    for c in range(2):
        e = _scaled_normal(rng, shape, 1.5)
        e[(0,) * l] -= goal[c]
        cost += poly_mul(e, e)
    return cost


def _shift_basis(svals, n):
    """For each shift s: the (n x n) matrix whose column j holds the coefficients
    of (q - s)^j (repeated multiplication by the linear factor q - s)."""
    svals = np.asarray(svals, dtype=np.float64)
    out = np.zeros((len(svals), n, n))
    col = np.zeros((len(svals), n))
    col[:, 0] = 1.0
    out[:, :, 0] = col
    for j in range(1, n):
        nxt = np.zeros_like(col)
        nxt[:, 1:] = col[:, :-1]          # times q
        nxt -= svals[:, None] * col       # times -s
        col = nxt
        out[:, :, j] = col
    return out


def _obstacle_constraints(rng, l: int, deg: int, count: int, q0) -> list:
    """FRS-like obstacle constraints: one template T of multi-degree (deg,)*l,
    shifted by s_i = o_i/2 for obstacle points o_i uniform in a 4 m x 4 m window
    (extra axes shifted uniformly in [-1,1]), then planted feasible at q0:
    g_i(q) = T(q - s_i) - T(q0 - s_i) - U(0.1, 0.5)."""
    tmpl = _scaled_normal(rng, (deg + 1,) * l, 1.5)
    shifts = np.empty((count, l))
    margins = np.empty(count)
    for i in range(count):   # the draws stay in the order of one constraint at a time
        o = rng.uniform(-2.0, 2.0, size=2)
        shifts[i] = np.concatenate([o / 2.0, rng.uniform(-1.0, 1.0, size=l - 2)])
        margins[i] = rng.uniform(0.1, 0.5)
    m = deg + 1
    coef = np.broadcast_to(tmpl, (count,) + tmpl.shape).copy()
    for k in range(l):
        B = _shift_basis(shifts[:, k], m)                     # (count, m, m)
        moved = np.moveaxis(coef, k + 1, 1)                   # (count, m, ...)
        moved = np.einsum("cab,cb...->ca...", B, moved)
        coef = np.moveaxis(moved, 1, k + 1)
    at_q0 = poly_eval_many(tmpl, np.asarray(q0)[None, :] - shifts)
    coef[(slice(None),) + (0,) * l] -= at_q0 + margins
    return [np.ascontiguousarray(c) for c in coef]


# ---- the RTD planning problem (Sec. II-C, Sec. VI) --------------------------------------
#
# A plan q = (q1, q2) in Q = [0,1] x [-1,1] drives the robot from the origin,
# heading along +x, at speed V_MAX q1 with yaw rate W_MAX q2 for T_PLAN
# seconds (a unicycle).  The FRS of Sec. II-C holds every (x, q) with x on the
# path of plan q, grown by the robot's radius and tracking error RHO.  RTD
# computes offline a polynomial w(x, q) that is >= 0 on the FRS (by sums of
# squares); here a stand-in is fitted instead: the least-squares polynomial
# of multi-degree (4, 4) in x and (10, 10) in q to the tube function
# s(x, q) = RHO^2 - min_t |x - path_q(t)|^2 on a Chebyshev grid, raised by a
# constant until it is >= 0 at every grid sample where s >= 0.  Online, each
# sensed obstacle point x_i gives the constraint w(x_i, q) + EPS_Q <= 0.

V_MAX, W_MAX, T_PLAN, RHO, EPS_Q = 1.0, 1.0, 1.5, 0.3, 1e-4
FRS_XDEG, FRS_QDEG = 4, 10
_FRS_CACHE = {}


def _unicycle_path(q1, q2, t):
    """Position at time t on the path of plan (q1, q2), arrays broadcast."""
    v, w = V_MAX * q1, W_MAX * q2
    small = np.abs(w) < 1e-9
    ws = np.where(small, 1.0, w)
    px = np.where(small, v * t, v * np.sin(w * t) / ws)
    py = np.where(small, 0.0, v * (1.0 - np.cos(w * t)) / ws)
    return px, py


def _cheb_nodes(n, a, b):
    k = np.arange(n)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos((2 * k + 1) * np.pi / (2 * n))


def frs_polynomial() -> np.ndarray:
    """Coefficients W[a, b, c, d] of the FRS-like w(x, q) = sum W x1^a x2^b q1^c q2^d
    (shape (5, 5, 11, 11)); deterministic (no random draws), computed once per
    process."""
    if "w" in _FRS_CACHE:
        return _FRS_CACHE["w"]
    nx, nq, nt = 24, 28, 61
    X1, X2 = _cheb_nodes(nx, -0.5, 2.0), _cheb_nodes(nx, -1.6, 1.6)
    Q1, Q2 = _cheb_nodes(nq, 0.0, 1.0), _cheb_nodes(nq, -1.0, 1.0)
    q1g, q2g, tg = np.meshgrid(Q1, Q2, np.linspace(0.0, T_PLAN, nt), indexing="ij")
    px, py = _unicycle_path(q1g, q2g, tg)
    S = np.empty((nx, nx, nq, nq))
    for a in range(nx):
        dx2 = (X1[a] - px) ** 2
        for b in range(nx):
            S[a, b] = RHO ** 2 - np.min(dx2 + (X2[b] - py) ** 2, axis=-1)
    axes = ((X1, FRS_XDEG), (X2, FRS_XDEG), (Q1, FRS_QDEG), (Q2, FRS_QDEG))
    V = [npp.polyvander(v, d) for v, d in axes]
    P = [np.linalg.pinv(m) for m in V]
    # least squares on a tensor grid: the pseudo-inverse of a Kronecker
    # product is the Kronecker product of the pseudo-inverses
    W = np.einsum("ia,jb,kc,ld,abcd->ijkl", P[0], P[1], P[2], P[3], S, optimize=True)
    fit = np.einsum("ai,bj,ck,dl,ijkl->abcd", V[0], V[1], V[2], V[3], W, optimize=True)
    W[0, 0, 0, 0] += max(0.0, float(np.max(-fit[S >= 0.0])))
    _FRS_CACHE["w"] = W
    return W


def rtd_constraints(W: np.ndarray, pts: np.ndarray, eps_q: float = EPS_Q) -> list:
    """g_i(q) = w(x_i, q) + eps_q for each obstacle point x_i (rows of pts):
    coefficient tensors in q, multi-degree (10, 10)."""
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 2)
    V1 = npp.polyvander(pts[:, 0], W.shape[0] - 1)
    V2 = npp.polyvander(pts[:, 1], W.shape[1] - 1)
    G = np.einsum("na,nb,abcd->ncd", V1, V2, W)
    G[:, 0, 0] += eps_q
    return [np.ascontiguousarray(g) for g in G]


def _box_outline(center, angle, half=0.15, step=0.05) -> np.ndarray:
    """Points every `step` metres along the outline of a square of side 2 half."""
    n = int(round(2 * half / step))
    s = np.linspace(-half, half, n + 1)[:-1]
    pts = np.concatenate([np.stack([s, np.full_like(s, -half)], 1), np.stack([np.full_like(s, half), s], 1),
                          np.stack([-s, np.full_like(s, half)], 1), np.stack([np.full_like(s, -half), -s], 1)])
    c, sn = math.cos(angle), math.sin(angle)
    return pts @ np.array([[c, -sn], [sn, c]]).T + np.asarray(center)


def endpoint_map() -> tuple:
    """The endpoint of plan q after T_PLAN as polynomials in q (multi-degree (1, 3)
    each): the unicycle's endpoint expanded to third order in the yaw rate."""
    a, b = V_MAX * T_PLAN, W_MAX * T_PLAN
    ex, ey = np.zeros((2, 4)), np.zeros((2, 4))
    ex[1, 0], ex[1, 2] = a, -a * b * b / 6.0
    ey[1, 1], ey[1, 3] = a * b / 2.0, -a * b ** 3 / 24.0
    return ex, ey


def rtd_pop(rng) -> tuple:
    """One planning iteration: obstacle points, the two waypoints, the cost."""
    nbox = int(rng.integers(2, 11))
    pts = []
    for _ in range(nbox):
        center = (rng.uniform(0.3, 3.0), rng.uniform(-1.2, 1.2))
        pts.append(_box_outline(center, rng.uniform(0.0, 0.5 * math.pi)))
    pts = np.concatenate(pts)
    # waypoints 1.5 m ahead, on the left and on the right of the hallway
    wps = [np.array([1.5, 0.5 + 0.1 * rng.standard_normal()]),
           np.array([1.5, -0.5 + 0.1 * rng.standard_normal()])]
    ex, ey = endpoint_map()
    cost = np.ones((1, 1))
    for xn in wps:
        dxp, dyp = ex.copy(), ey.copy()
        dxp[0, 0] -= xn[0]
        dyp[0, 0] -= xn[1]
        cost = poly_mul(cost, poly_mul(dxp, dxp) + poly_mul(dyp, dyp))
    return pts, wps, cost


def make_instance(config: int, index: int = 0, **overrides) -> Instance:
    """Instance `index` of workload `config` (0..6), seeded PCG64(1_000_003*c + k)."""
    rng = np.random.Generator(np.random.PCG64(SEED_STRIDE * config + index))
    if config == 0:
        l = 2
        cost = rng.standard_normal((5, 5))
        q0 = rng.uniform(-1.0, 1.0, size=l)
        ineq = [_planted(rng, _scaled_normal(rng, (5, 5), 2.0), q0) for _ in range(16)]
        inst = Instance("small", l, -np.ones(l), np.ones(l), cost, ineq, [],
                        max_boxes=1 << 16, q0=q0)
    elif config == 1:
        l = 2
        q0 = rng.uniform(-1.0, 1.0, size=l)
        cost = _goal_cost(rng, l, 3)
        ineq = _obstacle_constraints(rng, l, 10, 500, q0)
        inst = Instance("rtd", l, -np.ones(l), np.ones(l), cost, ineq, [],
                        max_boxes=1 << 20, q0=q0)
    elif config == 2:
        l = 4
        q0 = rng.uniform(-1.0, 1.0, size=l)
        cost = _scaled_normal(rng, (5,) * l, 2.0)
        ineq = [_planted(rng, _scaled_normal(rng, (5,) * l, 2.0), q0) for _ in range(100)]
        eq = []
        for _ in range(2):
            h = _scaled_normal(rng, (3,) * l, 2.0)
            h[(0,) * l] -= poly_eval(h, q0)
            eq.append(h)
        inst = Instance("4d", l, -np.ones(l), np.ones(l), cost, ineq, eq,
                        max_boxes=1 << 20, q0=q0)
    elif config in (3, 4):
        if config == 3:
            l = int(rng.integers(2, 4))
            deg = int(rng.choice([4, 6, 8, 10]))
            count = int(round(math.exp(rng.uniform(math.log(50), math.log(1000)))))
        else:
            l, deg = 2, 10
            count = int(round(math.exp(rng.uniform(math.log(100), math.log(2000)))))
        q0 = rng.uniform(-1.0, 1.0, size=l)
        cost = _goal_cost(rng, l, 3)
        ineq = _obstacle_constraints(rng, l, deg, count, q0)
        inst = Instance("batch" if config == 3 else "serve", l, -np.ones(l), np.ones(l),
                        cost, ineq, [], max_boxes=1 << 20, q0=q0)
    elif config == 5:
        # a plan through waypoints (the multi-waypoint cost of Sec. VI): the
        # product over two waypoints x_n of the squared distance of the
        # endpoint map e(q) (multi-degree (3,3) per component) from x_n, which
        # has a minimum near each waypoint's preimage; 100 obstacle
        # constraints (10,10) as in the rtd workload
        l = 2
        q0 = rng.uniform(-1.0, 1.0, size=l)
        e = [_scaled_normal(rng, (4, 4), 1.5) for _ in range(2)]
        cost = np.ones((1, 1))
        for _ in range(2):
            xn = rng.uniform(-2.0, 2.0, size=2)
            d = np.zeros((7, 7))
            for c in range(2):
                ec = e[c].copy()
                ec[0, 0] -= xn[c]
                d += poly_mul(ec, ec)
            cost = poly_mul(cost, d)
        ineq = _obstacle_constraints(rng, l, 10, 100, q0)
        inst = Instance("waypoints", l, -np.ones(l), np.ones(l), cost, ineq, [],
                        max_boxes=1 << 20, q0=q0)
    elif config == 6:
        pts, _, cost = rtd_pop(rng)
        ineq = rtd_constraints(frs_polynomial(), pts)
        inst = Instance("rtdpop", 2, np.array([0.0, -1.0]), np.array([1.0, 1.0]), cost, ineq, [],
                        max_boxes=1 << 20)
    else:
        raise ValueError(f"unknown workload {config}")
    if overrides:
        inst = inst.with_options(**overrides)
    return inst


def truncate(inst: Instance, n_ineq: int | None = None, n_eq: int | None = None) -> Instance:
    """Same instance with only the first n_ineq / n_eq constraints (smaller test cases)."""
    return dataclasses.replace(
        inst,
        ineq=inst.ineq[: (len(inst.ineq) if n_ineq is None else n_ineq)],
        eq=inst.eq[: (len(inst.eq) if n_eq is None else n_eq)])
