"""FP64 CPU oracle for array BP-XOR coded matrix multiplication.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only the test-suite, the smoke check of the
entry module and the CPU-baseline leg of the benchmark may import it; the
product path (the C ABI library and its Python binding) never does, and this
package imports nothing from the product path.

Everything here is written from the paper (Arslan, "Array BP-XOR Codes for
Hierarchically Distributed Matrix Multiplication", arXiv 1904.11563):

* ``splitmix``  - the SplitMix64 counter-based generator (Steele, Lea and
                  Flood, OOPSLA 2014), used by the array-code search.
* ``codes``     - code objects: the array BP-XOR codes of Table I and
                  Table III, a deterministic search for array codes at
                  parameters the paper gives no construction for, and the
                  Mojette (projection-geometry) asymptotic codes of
                  Constructions A and B with their closed forms.
* ``peeling``   - BP (peeling) decoding of Sec. I-A over a set of received
                  symbols, the arrival prefix and the release schedule.
* ``pipeline``  - encode, coded products, numeric peel and the uncoded
                  product, all in float64.
* ``pipeline2d``- the two-dimensional form of Examples 1 and 2 (A split by
                  rows and B by columns, information symbols a_r b_c, gray
                  symbols), float64.

Parity status of each function is stated in its docstring; every function is
pinned by a test under ``tests/`` against facts the paper or mathematics fixes.
"""
