"""Differential compression of a binary coupling matrix (Sec. III.C, Alg. 2),
written out plainly with Python sets.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU-baseline
leg; never by the product path, and it shares no code with it.

The coupling matrix L has L_ij = 1 when element j influences element i; row i
is the set of positions j of its set bits.  Readings used where the paper
leaves a detail open:
  * a circular shift of a row "by i positions left" moves the bit at position
    p to position (p - i) mod n, so that a translation-invariant topology (row
    i = row 0 moved by i) shifts back onto row 0; the shift right is the
    inverse, p -> (p + i) mod n;
  * the common vector V is row 0 as given; every row, row 0 included, is
    compared with it, so row 0 always maps to the empty difference vector;
  * the difference table keeps its entries in order of first appearance as i
    runs upwards, and FIND returns the entry equal to d (entries are distinct).

compress() returns (V, D, C): V the sorted positions of the common vector, D
the list of difference vectors (each a sorted list of positions), C[i] the
index into D of row i.  extract() is the paper's EXTRACT for one row.
parity: pinned by tests/test_oracle_pins.py (the paper's full-mesh and ring
statements, round trips on random and structured matrices, the number of
entries of a periodic lattice against a count of its boundary patterns).
"""
import numpy as np


def rol(bits, i, n):
    """Circular shift left by i: position p -> (p - i) mod n."""
    return {(p - i) % n for p in bits}


def ror(bits, i, n):
    """Circular shift right by i: position p -> (p + i) mod n."""
    return {(p + i) % n for p in bits}


def rows_of(n, row_ptr, col):
    """Rows of a matrix given as CSR (row i lists the j with L_ij = 1) as sets."""
    rows = []
    for i in range(n):
        r = set(int(j) for j in col[row_ptr[i]:row_ptr[i + 1]])
        assert len(r) == row_ptr[i + 1] - row_ptr[i], "a row lists a position twice"
        rows.append(r)
    return rows


def compress(n, row_ptr, col):
    """COMPRESS of Alg. 2 on the rows of an n x n binary matrix."""
    rows = rows_of(n, row_ptr, col)
    V = set(rows[0])
    D, index, C = [], {}, []
    for i in range(n):
        d = rol(rows[i], i, n) ^ V  # XOR of bit vectors = symmetric difference of position sets
        key = tuple(sorted(d))
        if key not in index:  # FIND; append a new entry when absent
            index[key] = len(D)
            D.append(list(key))
        C.append(index[key])
    return sorted(V), D, np.array(C, dtype=np.int64)


def extract(i, n, V, D, C):
    """EXTRACT of Alg. 2: row i = ROR(XOR(V, D[C_i]), i), as sorted positions."""
    return sorted(ror(set(V) ^ set(D[C[i]]), i, n))


def extract_all(n, V, D, C):
    """Every row, as CSR (row_ptr int64, col int32, each row ascending)."""
    rp = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for i in range(n):
        r = extract(i, n, V, D, C)
        cols.extend(r)
        rp[i + 1] = rp[i] + len(r)
    return rp, np.array(cols, dtype=np.int32)
