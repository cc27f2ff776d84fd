"""IPFASST with multigrid node solves on AMD MI355X (gfx950).

The compute path is the HIP library ``libpfmg.so`` behind the C-ABI in
``include/pfmg.h``; ``pfmg`` is its thin Python binding.
"""
__all__ = ["pfmg"]
