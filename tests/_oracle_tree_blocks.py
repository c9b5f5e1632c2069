"""Helper for tests: the oracle's tree as (perm, blocks) arrays in the library's
get_tree layout (row_begin, row_end, col_begin, col_end, admissible)."""
import numpy as np

from oracle.geometry import Panels
from oracle.tree import ClusterTree, block_tree


def oracle_tree(xyz, tri, leaf, eta):
    P = Panels(xyz, tri)
    T = ClusterTree(P, leaf)
    B = block_tree(T, eta)
    blocks = np.array([(T.begin[a], T.end[a], T.begin[b], T.end[b], int(adm)) for a, b, adm in B],
                      dtype=np.int64).reshape(-1, 5)
    return P, T, B, T.perm.astype(np.int64), blocks
