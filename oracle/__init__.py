"""CPU oracle for the filtered Paterson-Stockmeyer matrix power series.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and
shares no code with it.

Contents:
  * ``fps_oracle.c`` (built to ``liboracle.so`` by ``oracle/build.py``):
    filtered and unfiltered PS (paper eqs. 2-6, 11, 13, 14; Algorithm 2 with a
    fixed entry threshold), single filtered products and coefficient sums,
    and a long-double dense Horner evaluation of the plain polynomial (eq. 1).
  * ``oracle.py``: ctypes wrapper, dense double Horner (eq. 1 by the Qin
    scheme, numpy matmul as the product step), norms.
  * series mode (Algorithm 2 steps 1-3): the 1-norm estimator on Z^p,
    the norm bounds of eq. 37 (Lemma 1), the degree N of eq. 34.
  * ``bound.py``: the paper's a-posteriori filtering error bound
    (eqs. 21-26 combined in eq. 23).
"""

from .oracle import (  # noqa: F401
    axpy,
    dense_horner,
    dense_horner_ld,
    filtered_ps,
    fro_norm,
    norm1,
    schedule,
    spgemm,
    unfiltered_ps,
    lib_path,
    alg1_filter,
    fnt_thresholds,
    filtered_ps_adaptive,
    normest1_power,
    power_norm_bounds,
    series_degree,
    series,
)
from .bound import filtering_bound, power_norms  # noqa: F401
