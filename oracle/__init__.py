"""Plain FP64 CPU oracle for the boundary Dirichlet-to-Neumann (DtN) operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package: only
the tests, the smoke check and the benchmark's CPU-baseline leg may call it.
It shares no code with the GPU path (no kernels, headers, index maps or
helpers); the only common dependency is the seeded input module `workloads`.

What it computes (Gillman & Martinsson, "An O(N) algorithm for constructing
the solution operator to 2D elliptic boundary value problems in the absence of
body loads"):

* `assemble`     - the five-point finite-difference system of Section 7 on an
                   n x n grid, scaled by h^2, with the boundary ring kept as
                   unknowns whose rows are one-sided normal differences
                   (reading R1, see `assemble.py`).
* `brute_dtn`    - the Schur complement of Section 3.1 of the whole grid onto
                   the boundary ring, by a dense solve (tiny grids).
* `sparse_apply` - the same operator applied to Dirichlet data through one
                   sparse direct solve of the full system (any grid).
* `solution_apply` - the solution operator G = S'^{-1} (Section 7) applied
                   through one sparse direct solve of the full system.
* `nd_dtn`       - the nested-dissection build of Section 3.3: quadtree of
                   Section 2, leaf Schur complements (Section 3.1, banded
                   interior solve), pairwise merges of Section 3.2.
* `dst_dtn`      - closed form of the operator for constant d and b = c = 0
                   by separation of variables (discrete sine modes).
* `hbs`          - reference ranks / compression of off-diagonal blocks
                   (Section 4, Section 6 Step 2) by column-pivoted QR.

Floating point is IEEE float64 throughout (numpy / LAPACK), except `dst_dtn`
which can evaluate in numpy.longdouble.
"""
from .grid import ring_nodes, ring_index_of, build_tree, box_ring, box_interior, Box
from .assemble import assemble
from .schur import brute_dtn, sparse_apply, schur_complement, solution_apply
from .nd import nd_dtn, leaf_schur, merge_pair, SingularError
from .closed_forms import dst_dtn, trace_on_ring
from . import hbs
from .body import body_operator, body_nested

__all__ = [
    "ring_nodes", "ring_index_of", "build_tree", "box_ring", "box_interior", "Box",
    "assemble", "brute_dtn", "sparse_apply", "schur_complement", "solution_apply",
    "nd_dtn", "leaf_schur", "merge_pair", "SingularError",
    "dst_dtn", "trace_on_ring", "hbs",
]
