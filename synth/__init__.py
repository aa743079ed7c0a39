"""Seeded synthetic inputs for the two-level nonlinear Schwarz solver.

This module produces *inputs only*: meshes, element partitions, boundary node
lists, coefficient fields and load samples.  It holds none of the solver's
arithmetic (no element integrals, no overlap construction, no Schwarz step),
so that the FP64 CPU oracle and the HIP path can both consume it without
sharing any of the method.

Problem statements (the paper, Section 1):
  * nonlinear diffusion  -div((u^2+1) grad u) = f on a rectangle, u = 0 on the
    boundary (eq. 1; the paper takes f = 1 on the unit square);
  * the mesh is a regular grid of squares, each split into two triangles
    along the (i,j)-(i+1,j+1) diagonal, counter-clockwise vertex order;
  * subdomains are boxes of whole grid cells (the paper partitions the dual
    graph of the mesh, i.e. by elements; Section 2, last paragraph).

Load data enter as samples of f at the three edge midpoints of every
element, ordered (v0,v1), (v1,v2), (v2,v0); each consumer integrates them.
The coefficient field enters as one value per element.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "p1_grid", "even_cuts", "box_partition", "boundary_nodes",
    "edge_midpoints", "fourier_modes", "fourier_eval", "rff_field",
    "rff_eval", "diffusion_case", "config1", "config2", "config4_instance",
    "config4", "concat_cases", "small_case", "mlp_init", "mlp_batch",
    "epoch_orders", "q1_grid", "seeded_cuts", "elasticity_case", "config3",
    "small_elasticity_case",
]


def p1_grid(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0):
    """Structured P1 triangulation of [0,lx]x[0,ly] with nx*ny cells.

    Node (i,j) has index g = j*(nx+1) + i and coordinates (i*lx/nx, j*ly/ny).
    Cell (i,j) yields two triangles, element 2*(j*nx+i) = [(i,j),(i+1,j),
    (i+1,j+1)] and element 2*(j*nx+i)+1 = [(i,j),(i+1,j+1),(i,j+1)].
    """
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    X, Y = np.meshgrid(i * (lx / nx), j * (ly / ny))
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny))
    ci = ci.ravel()
    cj = cj.ravel()
    n00 = cj * (nx + 1) + ci
    n10 = n00 + 1
    n11 = n00 + (nx + 1) + 1
    n01 = n00 + (nx + 1)
    conn = np.empty((2 * nx * ny, 3), dtype=np.int32)
    conn[0::2] = np.stack([n00, n10, n11], axis=1)
    conn[1::2] = np.stack([n00, n11, n01], axis=1)
    return xy, conn


def even_cuts(n_cells: int, n_boxes: int) -> np.ndarray:
    """Cut positions 0 = c_0 < ... < c_n = n_cells splitting cells evenly."""
    return np.array([(k * n_cells) // n_boxes for k in range(n_boxes + 1)],
                    dtype=np.int64)


def box_partition(nx: int, ny: int, cuts_x, cuts_y) -> np.ndarray:
    """Element -> subdomain map for box partitions of a p1_grid mesh.

    Box (bx,by) covers cells cuts_x[bx] <= i < cuts_x[bx+1],
    cuts_y[by] <= j < cuts_y[by+1] and has id bx + (len(cuts_x)-1)*by.
    Both triangles of a cell belong to the cell's box.
    """
    cuts_x = np.asarray(cuts_x)
    cuts_y = np.asarray(cuts_y)
    bx_of_i = np.searchsorted(cuts_x, np.arange(nx), side="right") - 1
    by_of_j = np.searchsorted(cuts_y, np.arange(ny), side="right") - 1
    nbx = len(cuts_x) - 1
    cell_box = (by_of_j[:, None] * nbx + bx_of_i[None, :]).ravel()
    return np.repeat(cell_box, 2).astype(np.int32)


def boundary_nodes(nx: int, ny: int, sides=("left", "right", "bottom", "top")):
    """Indices of p1_grid nodes lying on the chosen sides of the rectangle."""
    i, j = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    i = i.ravel()
    j = j.ravel()
    mask = np.zeros(i.shape, dtype=bool)
    if "left" in sides:
        mask |= i == 0
    if "right" in sides:
        mask |= i == nx
    if "bottom" in sides:
        mask |= j == 0
    if "top" in sides:
        mask |= j == ny
    return np.nonzero(mask)[0].astype(np.int64)


def edge_midpoints(xy: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """(E,3,2) midpoints of the element edges (v0,v1), (v1,v2), (v2,v0)."""
    p = xy[conn]
    return 0.5 * np.stack([p[:, 0] + p[:, 1], p[:, 1] + p[:, 2],
                           p[:, 2] + p[:, 0]], axis=1)


def fourier_modes(seed: int, n_modes: int = 8, amp: float = 10.0,
                  kmax: int = 8):
    """Amplitudes a ~ U(0,amp) and integer wave numbers k, l ~ U{1..kmax}.

    Drawn with NumPy's PCG64 in the order a, k, l.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0.0, amp, size=n_modes)
    k = rng.integers(1, kmax + 1, size=n_modes)
    l = rng.integers(1, kmax + 1, size=n_modes)
    return a, k, l


def fourier_eval(pts: np.ndarray, modes) -> np.ndarray:
    """f(x,y) = sum_m a_m sin(pi k_m x) sin(pi l_m y) at points (...,2)."""
    a, k, l = modes
    x = pts[..., 0][..., None]
    y = pts[..., 1][..., None]
    return np.sum(a * np.sin(np.pi * k * x) * np.sin(np.pi * l * y), axis=-1)


def rff_field(seed: int, n_features: int = 512, corr_len: float = 0.1):
    """Random Fourier features of a unit-variance squared-exponential field.

    Frequencies omega ~ N(0, corr_len^-2 I), phases ~ U(0, 2 pi).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = rng.normal(0.0, 1.0 / corr_len, size=(n_features, 2))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_features)
    return omega, phase


def rff_eval(pts: np.ndarray, field) -> np.ndarray:
    """g(x) = sqrt(2/M) sum_m cos(omega_m . x + phase_m) at points (...,2).

    Points on few distinct x and y values (grid centroids) use the identity
    cos(a + b) = cos a cos b - sin a sin b, which turns the sum into one
    small matrix product over the distinct coordinates.
    """
    omega, phase = field
    pts = np.asarray(pts, dtype=np.float64)
    shape = pts.shape[:-1]
    p2 = pts.reshape(-1, 2)
    xs, ix = np.unique(p2[:, 0], return_inverse=True)
    ys, iy = np.unique(p2[:, 1], return_inverse=True)
    scale = np.sqrt(2.0 / len(phase))
    if len(xs) * len(ys) <= 4 * len(p2) and len(xs) * len(ys) <= 2 ** 24:
        ax = np.outer(xs, omega[:, 0])
        by = np.outer(ys, omega[:, 1]) + phase
        grid = np.cos(ax) @ np.cos(by).T - np.sin(ax) @ np.sin(by).T
        return (scale * grid[ix, iy]).reshape(shape)
    arg = p2 @ omega.T + phase
    return (scale * np.cos(arg).sum(axis=-1)).reshape(shape)


def diffusion_case(nx, ny, cuts_x, cuts_y, overlap, *, two_level=False,
                   forcing=None, coef_field=None, beta=1.0, name="diffusion"):
    """Assemble the input dictionary of one diffusion problem.

    forcing:    None (f = 1) or a callable f(points) -> values.
    coef_field: None (kappa = 1) or a callable g(points); kappa_e = exp(g) at
                the element centroid.
    beta:       nonlinearity scale, coefficient (1 + beta u^2); beta = 0 gives
                the linear problem used by the reduction tests.
    """
    xy, conn = p1_grid(nx, ny)
    part = box_partition(nx, ny, cuts_x, cuts_y)
    bnd = boundary_nodes(nx, ny)
    elem_load = None
    if forcing is not None:
        elem_load = np.ascontiguousarray(forcing(edge_midpoints(xy, conn)))
    elem_coef = None
    if coef_field is not None:
        cen = xy[conn].mean(axis=1)
        elem_coef = np.exp(coef_field(cen))
    return {
        "name": name,
        "kind": "diffusion",
        "nx": nx, "ny": ny,
        "xy": xy, "conn": conn,
        "elem_part": part,
        "n_sub": (len(cuts_x) - 1) * (len(cuts_y) - 1),
        "overlap": int(overlap),
        "dirichlet": bnd,
        "dirichlet_vals": np.zeros(len(bnd)),
        "elem_load": elem_load,
        "elem_coef": elem_coef,
        "beta": float(beta),
        "two_level": bool(two_level),
    }


def config1():
    """64x64 P1 grid on the unit square, 4x4 boxes, overlap 1, f = 1,
    one-level (the paper's diffusion problem at small scale)."""
    return diffusion_case(64, 64, even_cuts(64, 4), even_cuts(64, 4), 1,
                          two_level=False, name="diffusion_64x64_4x4_ov1")


def config2(seed: int = 2):
    """512x512 P1 grid, 16x16 boxes, overlap 2, two-level, f a seeded sum
    of 8 Fourier modes with amplitudes U(0,10)."""
    modes = fourier_modes(seed)
    return diffusion_case(512, 512, even_cuts(512, 16), even_cuts(512, 16), 2,
                          two_level=True,
                          forcing=lambda p: fourier_eval(p, modes),
                          name="diffusion_512x512_16x16_ov2_gdsw")


def config4_instance(b: int):
    """One instance of the batched diffusion workload: grid n x n with
    n ~ U{128..384}, k x k boxes with k ~ U{8..16}, overlap 2, two-level,
    coefficient exp(g) with g a unit-variance random field (length 0.1)."""
    rng = np.random.Generator(np.random.PCG64(4000 + b))
    n = int(rng.integers(128, 385))
    k = int(rng.integers(8, 17))
    field = rff_field(4000 + b)
    return diffusion_case(n, n, even_cuts(n, k), even_cuts(n, k), 2,
                          two_level=True,
                          coef_field=lambda p: rff_eval(p, field),
                          name=f"diffusion_batch_{b}_{n}x{n}_{k}x{k}")


def concat_cases(cases, name="batch"):
    """Join independent problems into one disconnected mesh: node, element
    and subdomain indices of case b are offset by those of cases 0..b-1.
    All cases must agree on overlap and two_level; beta must be equal."""
    xy, conn, part, dn, dv, fl, kc = [], [], [], [], [], [], []
    n_off = e_off = s_off = 0
    for c in cases:
        xy.append(c["xy"])
        conn.append(c["conn"] + n_off)
        part.append(c["elem_part"] + s_off)
        dn.append(c["dirichlet"] + n_off)
        dv.append(c["dirichlet_vals"])
        E = len(c["conn"])
        fl.append(c["elem_load"] if c["elem_load"] is not None else np.ones((E, 3)))
        kc.append(c["elem_coef"] if c["elem_coef"] is not None else np.ones(E))
        n_off += len(c["xy"])
        e_off += E
        s_off += c["n_sub"]
    return {
        "name": name, "kind": "diffusion",
        "xy": np.concatenate(xy), "conn": np.concatenate(conn).astype(np.int32),
        "elem_part": np.concatenate(part).astype(np.int32), "n_sub": s_off,
        "overlap": cases[0]["overlap"],
        "dirichlet": np.concatenate(dn), "dirichlet_vals": np.concatenate(dv),
        "elem_load": np.concatenate(fl), "elem_coef": np.concatenate(kc),
        "beta": cases[0]["beta"], "two_level": cases[0]["two_level"],
        "instances": [(len(c["xy"]), c["name"]) for c in cases],
    }


def config4(n_instances: int = 32):
    """The batch of independent diffusion solves as one disconnected mesh."""
    return concat_cases([config4_instance(b) for b in range(n_instances)],
                        name=f"diffusion_batch_{n_instances}_grf")


def small_case(n=12, boxes=3, overlap=1, two_level=False, beta=1.0,
               forcing_seed=None, coef_seed=None, uneven=False):
    """Small diffusion problems for oracle pins and parity tests."""
    cx = even_cuts(n, boxes)
    cy = even_cuts(n, boxes)
    if uneven:
        # shift interior cuts to make the boxes unequal and the tail ragged
        cx = cx.copy()
        cy = cy.copy()
        cx[1:-1] = np.maximum(cx[1:-1] - 1, np.arange(1, boxes))
        cy[1:-1] = np.minimum(cy[1:-1] + 1, n - np.arange(boxes - 1, 0, -1))
    forcing = None
    if forcing_seed is not None:
        modes = fourier_modes(forcing_seed)
        forcing = lambda p: fourier_eval(p, modes)  # noqa: E731
    coef = None
    if coef_seed is not None:
        field = rff_field(coef_seed)
        coef = lambda p: rff_eval(p, field)  # noqa: E731
    return diffusion_case(n, n, cx, cy, overlap, two_level=two_level,
                          forcing=forcing, coef_field=coef, beta=beta,
                          name=f"small_{n}_{boxes}_{overlap}")


# ------------------------------------------------------ learned initial guess
def mlp_init(seed: int, dims=(320, 256, 256, 256, 256)) -> np.ndarray:
    """Initial network parameters, flat float32: for each affine layer the
    weights [out][in] row-major, then the biases, all ~ U(-1/sqrt(in),
    1/sqrt(in)) (PCG64, layer by layer, weights before biases)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l in range(len(dims) - 1):
        ni, no = dims[l], dims[l + 1]
        bound = 1.0 / np.sqrt(ni)
        parts.append(rng.uniform(-bound, bound, size=no * ni))
        parts.append(rng.uniform(-bound, bound, size=no))
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(seed: int, n: int, n_in: int = 320, n_out: int = 256):
    """A synthetic batch (inputs ~ N(0,1), targets ~ N(0,1)), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((n, n_in)).astype(np.float32)
    T = rng.standard_normal((n, n_out)).astype(np.float32)
    return X, T


def epoch_orders(seed: int, n: int, epochs: int) -> np.ndarray:
    """Sample order of every training epoch: `epochs` PCG64 permutations of
    range(n), concatenated, int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.concatenate([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)


# ------------------------------------------------------------ elasticity
def q1_grid(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0):
    """Structured Q1 mesh of [0,lx]x[0,ly] with nx*ny square cells.

    Node (i,j) has index g = j*(nx+1) + i; element j*nx+i has the nodes
    (i,j), (i+1,j), (i+1,j+1), (i,j+1) (counter-clockwise)."""
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    X, Y = np.meshgrid(i * (lx / nx), j * (ly / ny))
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny))
    n00 = (cj * (nx + 1) + ci).ravel()
    conn = np.stack([n00, n00 + 1, n00 + nx + 2, n00 + nx + 1], axis=1).astype(np.int32)
    return xy, conn


def _largest_remainder(w, total):
    q = w / w.sum() * total
    base = np.floor(q).astype(np.int64)
    rest = total - base.sum()
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rest]] += 1
    return base


def seeded_cuts(seed: int, nx: int, ny: int, nbx: int = 8, nby: int = 8,
                ratio=(2.0, 3.0)):
    """Box cuts at seeded positions: widths w ~ U(1, sqrt 3) per direction
    (x first, then y), scaled to whole cells by largest remainder; drawn
    again until the largest/smallest box area lies in [ratio[0], ratio[1]]
    (PCG64).  Returns (cuts_x, cuts_y)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    while True:
        wx = _largest_remainder(rng.uniform(1.0, np.sqrt(3.0), nbx), nx)
        wy = _largest_remainder(rng.uniform(1.0, np.sqrt(3.0), nby), ny)
        if wx.min() < 1 or wy.min() < 1:
            continue
        area = np.outer(wy, wx)
        r = area.max() / area.min()
        if ratio[0] <= r <= ratio[1]:
            return (np.concatenate([[0], np.cumsum(wx)]),
                    np.concatenate([[0], np.cumsum(wy)]))


def elasticity_case(nx, ny, lx, ly, cuts_x, cuts_y, overlap, *, E=210.0, nu=0.3,
                    traction=(0.0, -4.0), two_level=True, name="elasticity",
                    clamp_right=False, body=(0.0, 0.0)):
    """Compressible Neo-Hooke body on [0,lx]x[0,ly] with Q1 cells:
    x = 0 clamped (both dofs; with clamp_right also x = lx), traction t on
    the edge x = lx, lumped to nodal forces t * (edge length)/2 per node of
    every edge segment, and a volume force b as consistent nodal forces
    b * |cell| / 4 per node of every cell (the integral of each bilinear
    shape function over a rectangle).  Lame parameters from E, nu:
    mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu)).  Dofs are node-major,
    interleaved (u_x, u_y)."""
    xy, conn = q1_grid(nx, ny, lx, ly)
    cuts_x = np.asarray(cuts_x)
    cuts_y = np.asarray(cuts_y)
    bx = np.searchsorted(cuts_x, np.arange(nx), side="right") - 1
    by = np.searchsorted(cuts_y, np.arange(ny), side="right") - 1
    part = (by[:, None] * (len(cuts_x) - 1) + bx[None, :]).ravel().astype(np.int32)
    fixed = np.isclose(xy[:, 0], 0.0)
    if clamp_right:
        fixed |= np.isclose(xy[:, 0], lx)
    clamped = np.nonzero(fixed)[0]
    dofs = np.sort(np.concatenate([2 * clamped, 2 * clamped + 1])).astype(np.int64)
    right = np.nonzero(np.isclose(xy[:, 0], lx))[0]
    right = right[np.argsort(xy[right, 1])]
    f = np.zeros(2 * len(xy))
    hy = ly / ny
    for a, b in zip(right[:-1], right[1:]):
        for g in (a, b):
            f[2 * g] += traction[0] * hy / 2
            f[2 * g + 1] += traction[1] * hy / 2
    if body[0] != 0.0 or body[1] != 0.0:
        q = (lx / nx) * (ly / ny) / 4.0
        for comp in (0, 1):
            np.add.at(f, 2 * conn.ravel() + comp, body[comp] * q)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return {
        "name": name, "kind": "neohooke",
        "nx": nx, "ny": ny, "xy": xy, "conn": conn, "elem_part": part,
        "n_sub": (len(cuts_x) - 1) * (len(cuts_y) - 1), "overlap": int(overlap),
        "dirichlet": dofs, "dirichlet_vals": np.zeros(len(dofs)),
        "nodal_force": f, "mu": mu, "lam": lam, "E": E, "nu": nu,
        "two_level": bool(two_level),
    }


def config3(traction_max: float = 4.0):
    """256x128 Q1 cells on [0,2]x[0,1], 8x8 subdomains at seeded cuts (area
    ratio 2..3, seed 3), overlap 2, GDSW, E = 210, nu = 0.3, right-edge
    traction (0, -traction_max) at the last of the load steps."""
    cx, cy = seeded_cuts(3, 256, 128)
    return elasticity_case(256, 128, 2.0, 1.0, cx, cy, 2, traction=(0.0, -traction_max),
                           name="neohooke_256x128_8x8_ov2_gdsw")


def beam_case(force: float, nx: int = 320, ny: int = 64, boxes=(20, 4), overlap: int = 2,
              two_level: bool = True):
    """The paper's beam (Section 1 with eq. 2; Section 3): the rectangle
    [0,5]x[0,1], both ends clamped, volume force (0, -force), E = 210,
    nu = 0.3 (nondimensional), Q1 cells nx x ny, boxes[0] x boxes[1] box
    subdomains with the given overlap."""
    return elasticity_case(nx, ny, 5.0, 1.0, even_cuts(nx, boxes[0]), even_cuts(ny, boxes[1]),
                           overlap, traction=(0.0, 0.0), body=(0.0, -float(force)),
                           clamp_right=True, two_level=two_level,
                           name=f"beam_{nx}x{ny}_{boxes[0]}x{boxes[1]}_ov{overlap}_f{force:g}")


def small_elasticity_case(nx=8, ny=4, boxes=(2, 2), overlap=1, traction=(0.0, -1.0),
                          two_level=True, lx=2.0, ly=1.0):
    """Small cantilevers for oracle pins and parity tests."""
    return elasticity_case(nx, ny, lx, ly, even_cuts(nx, boxes[0]), even_cuts(ny, boxes[1]),
                           overlap, traction=traction, two_level=two_level,
                           name=f"small_nh_{nx}x{ny}_{boxes[0]}x{boxes[1]}_{overlap}")
