"""D3Q19 velocity set (Sec. 2.1, Fig. d3q19; Qian, d'Humieres and Lallemand 1992).

The paper shows the 19 directions only in a figure, so the numbering and the
weights are the standard ones of the cited D3Q19 model:

* alpha = 0 rest; 1-6 the axis directions +x,-x,+y,-y,+z,-z; 7-18 the twelve
  face diagonals in pairs (d, -d): (+x+y), (+x-y), (+x+z), (+x-z), (+y+z), (+y-z).
* w_0 = 1/3, w_1..6 = 1/18, w_7..18 = 1/36; lattice speed of sound c_s^2 = 1/3.
* The opposite of an odd alpha is alpha+1, of an even alpha >= 2 it is alpha-1.
"""
import numpy as np

Q = 19

E = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
], dtype=np.int64)

W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=np.float64)

OPP = np.array([0] + [a + 1 if a % 2 == 1 else a - 1 for a in range(1, Q)], dtype=np.int64)

# 36 * (2 w_alpha): integer weights of the geometric part 2 w_alpha e_alpha of the
# momentum-exchange term (4 on axis links, 2 on diagonal links).
TWO_W_36 = np.array([12] + [4] * 6 + [2] * 12, dtype=np.int64)
