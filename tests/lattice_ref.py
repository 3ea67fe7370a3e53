"""D2Q9 lattice retyped from Sec. 3 of arXiv 1911.12913 (velocity columns and
weights as printed), for tests that need closed forms independent of both
implementations."""
import numpy as np

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 9, 1 / 36, 1 / 36, 1 / 36, 1 / 36])
CS2 = 1.0 / 3.0
