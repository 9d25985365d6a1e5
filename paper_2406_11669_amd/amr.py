"""Nested mesh refinement over batched patches: box in box without subcycling.

The inter-level operators of Sec. 3.9 (asterx_prolong, asterx_restrict) tie a hierarchy of patches together, as
in the mesh-refinement test of Sec. 4 (an inner box at half the spacing, prolongation at its boundary): all
patches advance with one time step through the persistent batched launches (Batch), and

* after the recovery of every stage, the primitives in a refined patch's ghost zones are prolonged from its
  parent (after the parent's own ghosts are filled);
* after every stage output, the nine evolved fields in its ghost zones are prolonged from the parent's stage
  output, each with its staggering (conserved variables at centres, A_i on edges, Psi at vertices);
* after every step, the refined patch's owned points are restricted onto the parent points they cover (finest
  level first), and the ghost zones are filled again.

Subcycling in time is not described in the paper (its method is announced as unpublished), so every level takes
the finest level's step.  The ghost zones of a patch are six boxes around its owned points (full extent along
the axes already covered), one prolongation call per field and box on the batch pools' per-patch slices.
"""
from paper_2406_11669_amd import asterx as ax

# staggering of the nine evolved fields (per axis: 0 cell-centred, 1 vertex-centred)
STATE_STAG = [(0, 0, 0)] * 5 + [(0, 1, 1), (1, 0, 1), (1, 1, 0), (1, 1, 1)]
PRIM_STAG = [(0, 0, 0)] * 5


def ghost_boxes(layout, stag):
    """The ghost points of a field with staggering stag as six inclusive index boxes (lo, hi): ng layers on each
    side of the owned points [0, n - 1], i.e. indices [-ng, n - 1 + ng + stag_d] along axis d (a vertex-centred
    axis also has its point n beyond the owned ones)."""
    n, g = layout.n, layout.ng
    full = [(-g, n[d] - 1 + g + stag[d]) for d in range(3)]
    own = [(0, n[d] - 1) for d in range(3)]
    boxes = []
    for d in range(3):
        for lo_side in (True, False):
            lo, hi = [0, 0, 0], [0, 0, 0]
            for e in range(3):
                r = full[e] if e > d else (own[e] if e < d else None)
                if e == d:
                    r = (-g, -1) if lo_side else (n[d], full[d][1])
                lo[e], hi[e] = r
            boxes.append((tuple(lo), tuple(hi)))
    return boxes


def owned_box_in_parent(layout, c0):
    """Parent points covered by the child's owned points: [c0, c0 + n/2 - 1] along every axis and staggering."""
    return tuple(c0), tuple(c0[d] + layout.n[d] // 2 - 1 for d in range(3))


class BoxInBox(ax.Batch):
    """Batch of nested patches (workloads.box_in_box): parents[p] is patch p's parent (None for the root), c0[p]
    the parent vertex index of its vertex 0.  Parents must come before their children."""

    def __init__(self, workloads, parents, c0, tuning=(4, 1), device="cuda"):
        self.parents = list(parents)
        self.c0 = list(c0)
        for p, q in enumerate(self.parents):
            assert q is None or q < p, "parents must precede their children"
        super().__init__(workloads, tuning=tuning, device=device, fused=True)
        self.fill_state(self.state)

    def _field(self, pool, f, p):
        L = self.wls[p].layout
        o = self.off[p]
        return pool[f:f + 1, o:o + L.npts]

    def _prolong_ghosts(self, pool, stags):
        """Ghost zones of every refined patch, from its parent, for the fields of pool (one staggering each)."""
        for p, q in enumerate(self.parents):
            if q is None:
                continue
            Lc, Lf = self.wls[q].layout, self.wls[p].layout
            for f, st in enumerate(stags):
                src, dst = self._field(pool, f, q), self._field(pool, f, p)
                for lo, hi in ghost_boxes(Lf, st):
                    ax.prolong(Lc, Lf, self.c0[p], st, src, dst, lo, hi)

    def restrict_all(self, U):
        """Owned points of every refined patch onto its parent, finest level first."""
        for p in reversed(range(len(self.parents))):
            q = self.parents[p]
            if q is None:
                continue
            Lc, Lf = self.wls[q].layout, self.wls[p].layout
            lo, hi = owned_box_in_parent(Lf, self.c0[p])
            for f, st in enumerate(STATE_STAG):
                ax.restrict(Lc, Lf, self.c0[p], st, self._field(U, f, p), self._field(U, f, q), lo, hi)

    def fill_state(self, U):
        super().fill_state(U)
        self._prolong_ghosts(U, STATE_STAG)

    def recover(self, U):
        super().recover(U)
        self._prolong_ghosts(self.prim, PRIM_STAG)

    def step(self):
        super().step()
        self.restrict_all(self.state)
        self.fill_state(self.state)
