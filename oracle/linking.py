"""Linking number and writhe of closed DNA conformations: test infrastructure.

The oracle for the topology analytics of circular DNA (Sec. 4.2 and the
appendix on the closure procedure): the linking number of the two strands is
Gauss's double integral

    Lk(C_R, C_B) = 1/(4 pi) oint oint (r_R - r_B) . (dr_R x dr_B) / |r_R - r_B|^3

over the two closed strand curves, and the writhe of the centreline is the
same integral of the centreline with itself.  The paper evaluates the
integral by quadrature with three intermediate points between beads; on
polygons it has an exact value, the sum over segment pairs of the signed
solid angle that one segment subtends as seen from the other (Klenin and
Langowski, Biopolymers 54, 307 (2000)), which is what is computed here, in
FP64, with the asin form of that solid angle (each asin taken as an atan2 of
the sine and cosine of the angle between two unit normals).

`crossing_linking` and `directional_writhe` count signed crossings of a
planar projection instead: an independent route to the same numbers (the
Gauss map's degree), used to pin the solid-angle sums.

Curves: strand s of a replica is the closed polygon of its beads in bp
order; both strands are oriented along increasing bp index (the ribbon
convention: a relaxed right-handed duplex has Lk ~ +N/10).  The centreline
runs through the midpoints of the two patches of each base pair (Sec. 3.1).

Open (linear) duplexes are closed as the appendix describes: each strand
is extended from both ends along the tangent of its terminal pair of beads,
outwards, by a distance D, and the two far points are joined by a straight
closing segment; the linking number of the two closed strands follows from
the same integral.  D is ten contour lengths of the relaxed duplex
(10 x 0.34 nm per base pair) unless given.  The centreline of an open
duplex is not closed (a straight chain's closing segment would run back
along its own axis): its writhe is the integral over the pairs of segments
of the open polygon that share no vertex.

Only tests may import this module; it shares no code with the GPU path.
"""
import numpy as np


def ring_curves(bead, patch, off, n_bp):
    """Strand-0 beads, strand-1 beads and centreline points ([n_bp, 3] each)
    of the replica whose first nucleotide is `off` (bp-major order)."""
    b = np.asarray(bead, dtype=np.float64)[off:off + 2 * n_bp].reshape(n_bp, 2, 3)
    p = np.asarray(patch, dtype=np.float64)[off:off + 2 * n_bp].reshape(n_bp, 2, 3)
    return b[:, 0].copy(), b[:, 1].copy(), 0.5 * (p[:, 0] + p[:, 1])


RISE_NM = 0.34          # relaxed rise per base pair (Sec. 2)
CLOSURE_CONTOURS = 10.0  # extension length in contour lengths


def closure_length(n_bp):
    """Default extension length D of the closure of an n_bp duplex."""
    return CLOSURE_CONTOURS * RISE_NM * n_bp


def close_strand(b, D):
    """The closed polygon of an open strand's beads b [n, 3] (n >= 2):
    b_0 .. b_n-1, then b_n-1 + D t_end, then b_0 + D t_start (the closing
    segment joins these two; the last edge returns to b_0), with t_end and
    t_start the outward unit tangents of the terminal bead pairs."""
    b = np.asarray(b, dtype=np.float64)
    t_start = b[0] - b[1]
    t_end = b[-1] - b[-2]
    t_start = t_start / np.linalg.norm(t_start)
    t_end = t_end / np.linalg.norm(t_end)
    return np.vstack([b, (b[-1] + D * t_end)[None], (b[0] + D * t_start)[None]])


def open_writhe(C):
    """Writhe of the open polygon C [n, 3]: twice the sum over unordered
    pairs of its n - 1 segments that share no vertex (no closing segment)."""
    C = np.asarray(C, dtype=np.float64)
    n = len(C)
    total = 0.0
    for i in range(n - 3):
        j = np.arange(i + 2, n - 1)
        total += segment_pair_omega(C[i], C[i + 1], C[j], C[j + 1]).sum()
    return 2.0 * total / (4.0 * np.pi)


def replica_topology(bead, patch, off, n_bp, ring, D=None):
    """(Lk, Wr) of one replica: a ring's closed strands and centreline, or an
    open duplex's strands closed by the appendix's procedure and its open
    centreline (D: extension length, default closure_length(n_bp))."""
    A, B, C = ring_curves(bead, patch, off, n_bp)
    if ring:
        return linking_number(A, B), writhe(C)
    D = closure_length(n_bp) if D is None else D
    return linking_number(close_strand(A, D), close_strand(B, D)), open_writhe(C)


def _unit(x):
    return x / np.linalg.norm(x, axis=-1, keepdims=True)


def _unit_or_zero(x):
    n = np.linalg.norm(x, axis=-1, keepdims=True)
    return np.where(n > 0.0, x / np.where(n > 0.0, n, 1.0), 0.0)


def segment_pair_omega(p1, p2, p3, p4):
    """Signed solid angle of segment p3->p4 seen from segment p1->p2 (arrays
    of shape [..., 3]): the Gauss integral over the pair times 4 pi.

    Klenin & Langowski: with r_ij = p_j - p_i, the four unit normals
    n1 ~ r13 x r14, n2 ~ r14 x r24, n3 ~ r24 x r23, n4 ~ r23 x r13 give
    Omega* = sum of asin(n_k . n_k+1) round the quadrangle, and the sign
    is that of (r34 x r12) . r13."""
    r13, r14, r23, r24 = p3 - p1, p4 - p1, p3 - p2, p4 - p2
    # collinear segments span no solid angle: a vanishing normal counts 0
    n1 = _unit_or_zero(np.cross(r13, r14))
    n2 = _unit_or_zero(np.cross(r14, r24))
    n3 = _unit_or_zero(np.cross(r24, r23))
    n4 = _unit_or_zero(np.cross(r23, r13))

    def asin_dot(a, b):
        # asin(a.b) for unit a, b, as the angle of (|a x b|, a.b): exact to
        # rounding near a.b = +-1, where asin itself loses half the digits
        return np.arctan2(np.sum(a * b, axis=-1), np.linalg.norm(np.cross(a, b), axis=-1))

    om = asin_dot(n1, n2) + asin_dot(n2, n3) + asin_dot(n3, n4) + asin_dot(n4, n1)
    sgn = np.sign(np.sum(np.cross(p4 - p3, p2 - p1) * r13, axis=-1))
    return om * sgn


def linking_number(A, B):
    """Gauss linking number of the closed polygons A [n, 3] and B [m, 3]
    (vertex k joined to k+1, the last to the first)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    a0, a1 = A, np.roll(A, -1, axis=0)
    b0, b1 = B, np.roll(B, -1, axis=0)
    total = 0.0
    for i in range(len(A)):  # one row of segment pairs at a time
        total += segment_pair_omega(a0[i], a1[i], b0, b1).sum()
    return total / (4.0 * np.pi)


def writhe(C):
    """Writhe of the closed polygon C [n, 3]: the Gauss integral of the curve
    with itself, i.e. twice the sum over unordered pairs of segments that
    share no vertex (a segment and its neighbours are coplanar and
    contribute nothing)."""
    C = np.asarray(C, dtype=np.float64)
    n = len(C)
    c0, c1 = C, np.roll(C, -1, axis=0)
    total = 0.0
    for i in range(n):
        j = np.arange(i + 2, n)
        if i == 0:
            j = j[j != n - 1]
        if len(j):
            total += segment_pair_omega(c0[i], c1[i], c0[j], c1[j]).sum()
    return 2.0 * total / (4.0 * np.pi)


def _basis(v):
    v = np.asarray(v, dtype=np.float64)
    v = v / np.linalg.norm(v)
    t = np.array([1.0, 0.0, 0.0]) if abs(v[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = _unit(np.cross(v, t))
    return v, e1, np.cross(v, e1)


def _crossings(a0, a1, b0, b1, v):
    """Projected crossings of segment a0->a1 with each segment b0->b1 along
    the viewing direction v: (mask, height of a, height of b, tangent sign
    v.(ta x tb)) per b segment."""
    v, e1, e2 = _basis(v)
    P = lambda x: np.stack([x @ e1, x @ e2], axis=-1)
    da, db = a1 - a0, b1 - b0
    da2, db2, w = P(da), P(db), P(b0 - a0)
    cr = lambda x, y: x[..., 0] * y[..., 1] - x[..., 1] * y[..., 0]
    den = cr(da2, db2)
    ok = den != 0.0
    den = np.where(ok, den, 1.0)
    s = cr(w, db2) / den
    t = cr(w, da2) / den
    hit = ok & (s >= 0.0) & (s < 1.0) & (t >= 0.0) & (t < 1.0)
    ha = (a0 + s[..., None] * da) @ v
    hb = (b0 + t[..., None] * db) @ v
    sg = np.sign(np.cross(da, db) @ v)
    return hit, ha, hb, sg


def crossing_linking(A, B, v):
    """Linking number from one projection: the crossings where A lies above
    B as seen from direction v, each counted with sign(v . (t_A x t_B)) (the
    preimages of v under the Gauss map, with their orientation)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    a1, b1 = np.roll(A, -1, axis=0), np.roll(B, -1, axis=0)
    total = 0
    for i in range(len(A)):
        hit, ha, hb, sg = _crossings(A[i], a1[i], B, b1, v)
        total += int(np.sum(sg[hit & (ha > hb)]))
    return total


def directional_writhe(C, dirs, closed=True):
    """Signed self-crossing number of the polygon C seen from each direction
    in dirs [k, 3] (each crossing once, sign(v . (t_upper x t_lower))); its
    mean over the sphere is the writhe.  closed=False: the open polygon of
    its n - 1 segments."""
    C = np.asarray(C, dtype=np.float64)
    n = len(C)
    c1 = np.roll(C, -1, axis=0)
    m = n if closed else n - 1       # segments
    out = []
    for v in dirs:
        total = 0
        for i in range(m):
            hit, ha, hb, sg = _crossings(C[i], c1[i], C[:m], c1[:m], v)
            j = np.arange(m)
            adj = (j == i) | (j == (i + 1) % n) | (j == (i - 1) % n)
            total += int(np.sum(sg[hit & ~adj & (ha > hb)]))
        out.append(total)
    return np.array(out)
