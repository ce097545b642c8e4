"""Plain CPU oracle for the exact resultant / discriminant / gcd path.

THIS PACKAGE IS TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_1201_1548_amd``) never imports, calls or links anything here, and the
code here shares nothing with the HIP kernels: no helpers, no tables, no
constants. It is deliberately slow and written to be checked by eye against the
paper (Berberich, Emeliyanenko, Kobel, Sagraloff, "Exact Symbolic-Numeric
Computation of Planar Algebraic Curves"):

* ``zx``          -- dense polynomials over Z in one variable (Python ints).
* ``resultant``   -- the Sylvester matrix of Section 2 ("Resultants" paragraph)
                     and its determinant over Z[x] by fraction-free (Bareiss)
                     elimination; the discriminant-style resultant res(f, f_y; y)
                     of Section 3.1 (Project); res_x by exchanging the variables.
* ``gcd``         -- gcd in Z[x] (Euclid over Q, then content), the object the
                     modular gcd of Section 5.1 ("Computing gcds in Z[x]")
                     reconstructs; plus gcd over F_p for certificates.
* ``closed_forms``-- inputs whose resultant is known in closed form.
* ``squarefree``  -- Yun's square-free decomposition in Z[x].
* ``subresultants``-- principal subresultant coefficients (determinant
                     definition of Section 3.2.2), the chain S_i and the
                     bounds N^- and N^+ of the same section, and the
                     resultant Q = res(f_x, f_y; y).

Precision: all arithmetic is exact (Python's unbounded integers and
``fractions.Fraction``). Pins that tie this oracle to the mathematics rather
than to itself live in ``tests/test_oracle_*.py``.
"""
