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


def tree_arrays(T, B):
    """The oracle's partition in gcq_upload_cluster_tree's arrays."""
    son = np.stack([np.asarray(T.son0), np.asarray(T.son1)], axis=1).astype(np.int32)
    son[son < 0] = -1
    rows = np.array([a for a, _, _ in B], np.int32)
    cols = np.array([b for _, b, _ in B], np.int32)
    adm = np.array([int(x) for _, _, x in B], np.uint8)
    return (T.perm.astype(np.int32), np.asarray(T.begin, np.int32), np.asarray(T.end, np.int32),
            son, rows, cols, adm)
