"""MI355X-native per-patch hydro update (MOL + PLM + HLL-family flux + TVD-RK2).

Importing the package loads nothing: the GPU library binding lives in
:mod:`paper_0910_5547_amd.amr` and the seeded inputs in
:mod:`paper_0910_5547_amd.workloads`.
"""
