"""Replica patterns (s, offsets) of the fractals used by the tests.

Replica j is the j-th listed offset.  The Sierpinski triangle follows the
orientation in which cell (x, y) is a member iff x & y == 0; the paper's own
orientation (replicas at (0,0), (0,1), (1,1): top, middle, right) is its
mirror image.  Carpet and Vicsek replicas are listed row by row.
"""
TRIANGLE = (2, ((0, 0), (1, 0), (0, 1)))
TRIANGLE_PAPER = (2, ((0, 0), (0, 1), (1, 1)))
CARPET = (3, ((0, 0), (1, 0), (2, 0), (0, 1), (2, 1), (0, 2), (1, 2), (2, 2)))
VICSEK = (3, ((1, 0), (0, 1), (1, 1), (2, 1), (1, 2)))

ALL = {"triangle": TRIANGLE, "triangle_paper": TRIANGLE_PAPER, "carpet": CARPET, "vicsek": VICSEK}

SEEDS = (2201, 1, 77, 123456789)
