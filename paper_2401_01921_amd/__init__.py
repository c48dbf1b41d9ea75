"""Block-sparse U(1) tensor contraction and DMRG H_eff.psi on MI355X.

The compute path lives in the C-ABI library ``libbst.so`` (HIP for gfx950);
``paper_2401_01921_amd.bst`` is its ctypes binding and
``paper_2401_01921_amd.workloads`` generates seeded synthetic inputs.
"""
