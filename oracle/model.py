"""Loop-balance and Roofline model (oracle side; test infrastructure only).

Sect. 4 (loop balance): every fluid-node update loads and stores the 19 PDFs
(D_pdf = 2 * 19 * 8 B in double precision); each indirectly addressed node
adds D_idx = 18 * 4 B of adjacency indices. OS-NT always addresses
indirectly; the AA pattern only in the odd time step, so its average over two
steps carries half of D_idx. Sect. 4.1: with RIA only run heads load indices,
and every run costs one block-vector entry D_block = 4 B. Sect. 5.2: the
Roofline prediction is bandwidth divided by loop balance.
"""

D_PDF = 2 * 19 * 8
D_IDX = 18 * 4
D_BLOCK = 4


def b_osnt():
    return D_PDF + D_IDX


def b_aa():
    return D_PDF + D_IDX / 2


def b_osnt_r(runs, nodes):
    """OS-NT-R: index and block traffic only once per run."""
    r = runs / nodes
    return D_PDF + (D_IDX + D_BLOCK) * r


def b_aa_r(runs, nodes):
    """AA-R: index and block traffic once per run, in every other step."""
    r = runs / nodes
    return D_PDF + (D_IDX + D_BLOCK) * r / 2


def roofline_mflups(bandwidth_gbs, loop_balance):
    """Sect. 5.2: P = b / B_l, in MFLUP/s for b in GB/s and B_l in B/FLUP."""
    return bandwidth_gbs * 1e3 / loop_balance
