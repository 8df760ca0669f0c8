"""CPU oracle for the PilotANN GPU stage and its CPU hand-off stages.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path imports this package;
only the tests, the smoke check and the benchmark's CPU-baseline leg may call
it.  It is plain, slow and written to be checked against the paper by eye:
fp64 arithmetic, Python loops where the method loops, library primitives
(matmul, eigh, sort) only as whole steps.  It shares no code with the HIP/C++
library and imports nothing from it.

Section references are to the PilotANN paper (Multi-stage processing in
section 4.1, methodology details in 4.3, fast entry selection in section 5,
Algorithm 1 "ANNS by Greedy Search", Algorithm 2 "Tiled FES GPU Kernel",
Table 2 complexity, evaluation metric in section 6.1).

Functions without an independent pin are marked "parity unpinned" in their
docstrings.
"""

from .metric import as_f32, delta, delta_many, recall_at_k  # noqa: F401
from .projection import fit_projection, project  # noqa: F401
from .knn import exact_knn  # noqa: F401
from .sampling import sample_nodes, check_subgraph, csr_from_padded, padded_from_csr  # noqa: F401
from .entries import balanced_kmeans, route, select_entries  # noqa: F401
from .traverse import greedy_search  # noqa: F401
from .stages import gpu_stage, refine, final_traversal, pipeline  # noqa: F401
