"""Simplicial meshes of the paper's test domains (Sec. 4.1): the triangle,
the disc, the tetrahedron and the ball of circumradius 5 centred at the
origin.

Input generation only: node coordinates and cells (node index triples or
quadruples), shared by the oracle and the GPU path; none of the method's
arithmetic (edge coefficients, control volumes, link variables) is computed
here.  The meshes are built explicitly, without a Delaunay search, so they are exactly
reproducible: the triangle as its regular subdivision into equilateral
triangles, the disc as rings of nodes stitched in angle order, the
tetrahedron as its regular lattice of tetrahedra and octahedra, each
octahedron split at its centre, the ball by the tetrahedra of the
body-centred cubic lattice inside it.
"""
import numpy as np

RADIUS = 5.0
SQ3 = np.sqrt(3.0)


def triangle(k):
    """Omega_tri, the triangle with vertices (0, 5), (-5 sqrt3 / 2, -5 / 2),
    (5 sqrt3 / 2, -5 / 2), split into k^2 equilateral triangles of side
    5 sqrt3 / k.  Nodes (k + 1)(k + 2) / 2, row by row from the bottom side
    (node (i, j) = B + i/k (C - B) + j/k (A - B)).  Returns (xy, tri)."""
    if k < 1:
        raise ValueError("k >= 1")
    A = np.array([0.0, RADIUS])
    B = np.array([-RADIUS * SQ3 / 2, -RADIUS / 2])
    Cv = np.array([RADIUS * SQ3 / 2, -RADIUS / 2])
    index = {}
    pts = []
    for j in range(k + 1):
        for i in range(k + 1 - j):
            index[(i, j)] = len(pts)
            pts.append(B + (i / k) * (Cv - B) + (j / k) * (A - B))
    tris = []
    for j in range(k):
        for i in range(k - j):
            tris.append((index[(i, j)], index[(i + 1, j)], index[(i, j + 1)]))
            if i + j <= k - 2:
                tris.append((index[(i + 1, j)], index[(i + 1, j + 1)], index[(i, j + 1)]))
    return np.array(pts, dtype=np.float64), np.array(tris, dtype=np.int64)


def disc(k):
    """Omega_circ, the disc of radius 5: the centre and k rings, ring r of 6r
    nodes at radius 5 r / k equally spaced in angle from angle 0; ring 1 is
    joined to the centre by six triangles, and each further ring to the one
    inside it by a merge of the two rings in angle order (at equal angles the
    inner ring advances first: every angle then stays below 90 degrees, so
    the mesh is Delaunay with every circumcentre inside its triangle).
    Nodes 1 + 3k(k + 1), triangles 6k^2.  Returns (xy, tri)."""
    if k < 1:
        raise ValueError("k >= 1")
    pts = [(0.0, 0.0)]
    start = [0]
    for r in range(1, k + 1):
        start.append(len(pts))
        for t in range(6 * r):
            th = 2.0 * np.pi * t / (6 * r)
            pts.append((RADIUS * r / k * np.cos(th), RADIUS * r / k * np.sin(th)))
    tris = [(0, start[1] + t, start[1] + (t + 1) % 6) for t in range(6)]
    for r in range(2, k + 1):
        ni, no = 6 * (r - 1), 6 * r
        a = b = 0  # steps taken along the inner / outer ring
        while a < ni or b < no:
            inner, outer = start[r - 1] + a % ni, start[r] + b % no
            # compare the angles of the next node on each ring: (a+1)/ni vs (b+1)/no
            if b < no and (a >= ni or (b + 1) * ni < (a + 1) * no):
                tris.append((inner, outer, start[r] + (b + 1) % no))
                b += 1
            else:
                tris.append((inner, outer, start[r - 1] + (a + 1) % ni))
                a += 1
    return np.array(pts, dtype=np.float64), np.array(tris, dtype=np.int64)


# Omega_tet: the regular tetrahedron of circumradius 5 (Sec. 4.1)
TET_VERTICES = RADIUS * np.array([[0.0, 0.0, 1.0], [2 * np.sqrt(2) / 3, 0.0, -1 / 3],
                                  [-np.sqrt(2) / 3, np.sqrt(2 / 3), -1 / 3], [-np.sqrt(2) / 3, -np.sqrt(2 / 3), -1 / 3]])


def tetrahedron(k):
    """Omega_tet, the regular tetrahedron of circumradius 5, by its lattice of
    edge 1/k: nodes (i, j, l) = V0 + i/k (V1 - V0) + j/k (V2 - V0) + l/k
    (V3 - V0), i + j + l <= k, ordered by l, then j, then i; cells: the
    upward tetrahedra, the downward ones and the octahedra between them, each
    octahedron split into the eight tetrahedra that join its centre to its
    faces.  The centres are appended after the lattice nodes, in the order of
    their octahedra.  Nodes (k + 1)(k + 2)(k + 3) / 6 + (k - 1) k (k + 1) / 6,
    cells k (k + 1)(k + 2) / 6 + (k - 2)(k - 1) k / 6 + 8 (k - 1) k (k + 1) / 6.

    The split around a centre gives every edge a coefficient alpha >= 0 (the
    centre's edges see the octahedron's faces at acute angles, and its
    faces' edges see the centre at right angles); the split of an octahedron
    into four tetrahedra around one of its diagonals would give that
    diagonal a negative one (the opposite dihedral angle is the
    octahedron's, above 90 degrees), which can leave K-hat indefinite in a
    magnetic field.  Returns (xyz, tets)."""
    if k < 1:
        raise ValueError("k >= 1")
    V = TET_VERTICES
    index = {}
    pts = []
    for l in range(k + 1):
        for j in range(k + 1 - l):
            for i in range(k + 1 - l - j):
                index[(i, j, l)] = len(pts)
                pts.append(V[0] + (i / k) * (V[1] - V[0]) + (j / k) * (V[2] - V[0]) + (l / k) * (V[3] - V[0]))
    cells = []
    centres = []
    for l in range(k):
        for j in range(k - l):
            for i in range(k - l - j):
                def at(di, dj, dl):
                    return index[(i + di, j + dj, l + dl)]
                cells.append((at(0, 0, 0), at(1, 0, 0), at(0, 1, 0), at(0, 0, 1)))
                if i + j + l <= k - 2:
                    # the octahedron's three antipodal vertex pairs; each face
                    # takes one vertex of every pair
                    pairs = ((at(1, 0, 0), at(0, 1, 1)), (at(0, 1, 0), at(1, 0, 1)), (at(0, 0, 1), at(1, 1, 0)))
                    c = len(pts) + len(centres)
                    centres.append(np.mean([pts[v] for pr in pairs for v in pr], axis=0))
                    for a in range(2):
                        for b in range(2):
                            for d in range(2):
                                cells.append((c, pairs[0][a], pairs[1][b], pairs[2][d]))
                if i + j + l <= k - 3:
                    cells.append((at(1, 1, 0), at(1, 0, 1), at(0, 1, 1), at(1, 1, 1)))
    return np.array(pts + centres, dtype=np.float64).reshape(-1, 3), np.array(cells, dtype=np.int64)


def ball(m):
    """Omega_ball, the ball of radius 5, by the body-centred cubic lattice of
    spacing h = 10 / m: cube corners at h (i - M/2) per axis and cube centres
    half a step off in every axis, M = m + 2 cubes across; cells: the
    tetrahedra that join two neighbouring centres to an edge of the square
    face between their cubes (four per pair, all congruent, with dihedral
    angles of 60 and 90 degrees, so every edge coefficient is >= 0), kept
    when their centroid lies in the closed ball.  No node is moved: the mesh
    is the ball up to a staircase layer of thickness below h at the sphere
    (its volume within 0.3 % of the ball's from m = 16 on).  Nodes that lie
    in a kept cell, in lexicographic (z, y, x) order of their half-step
    coordinates.  Returns (xyz, tets)."""
    if m < 2:
        raise ValueError("m >= 2")
    h = 2.0 * RADIUS / m
    M = m + 2
    # half-step integer coordinates: corners even (0 ... 2M), centres odd
    q = np.arange(2 * M + 1)
    Z, Y, X = np.meshgrid(q, q, q, indexing="ij")
    parity = (X % 2 == Y % 2) & (Y % 2 == Z % 2)
    code = np.full(X.shape, -1, dtype=np.int64)
    key = np.stack([X[parity], Y[parity], Z[parity]], axis=1)       # lexicographic (z, y, x)
    code[parity] = np.arange(len(key))
    pos = (key - M) * (0.5 * h)
    c = np.arange(1, 2 * M, 2)                                          # centre coordinates
    cells = []
    for axis in range(3):
        # centre pairs (a, a + 2 e_axis) and the square between them, whose
        # corners are the centres' coordinates +- 1 in the other two axes
        u, v = [b for b in range(3) if b != axis]
        A = np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1).reshape(-1, 3)[:, ::-1]   # (x, y, z)
        A = A[A[:, axis] + 2 <= 2 * M - 1]
        B = A.copy()
        B[:, axis] += 2
        ring = [(-1, -1), (1, -1), (1, 1), (-1, 1)]
        for t in range(4):
            P, Q = A.copy(), A.copy()
            P[:, axis] += 1
            Q[:, axis] += 1
            P[:, u] += ring[t][0]
            P[:, v] += ring[t][1]
            Q[:, u] += ring[(t + 1) % 4][0]
            Q[:, v] += ring[(t + 1) % 4][1]
            idx = [code[W[:, 2], W[:, 1], W[:, 0]] for W in (A, B, P, Q)]
            cells.append(np.stack(idx, axis=1))
    cells = np.concatenate(cells)
    centroid = pos[cells].mean(axis=1)
    cells = cells[np.sum(centroid * centroid, axis=1) <= RADIUS * RADIUS]
    used = np.zeros(len(key), dtype=bool)
    used[cells.ravel()] = True
    renum = np.cumsum(used) - 1
    return pos[used].astype(np.float64), renum[cells].astype(np.int64)


def domain(name, k):
    """(coordinates, cells) of "tri", "circ", "tet" or "ball" at refinement k."""
    if name == "tri":
        return triangle(k)
    if name == "circ":
        return disc(k)
    if name == "tet":
        return tetrahedron(k)
    if name == "ball":
        return ball(k)
    raise ValueError(f"unknown domain {name!r}")
