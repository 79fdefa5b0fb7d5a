"""MI355X-native compressible D2V16 MRT finite-difference lattice Boltzmann
model (Chen, Xu, Zhang, Li) behind a C-ABI HIP library.

Submodules are imported on demand: `inputs` (seeded synthetic workloads),
`lbm` (binding of the C-ABI library), `autograd` (adjoint-backed
torch.autograd.Function), `batch` (batched persistent form and its tuner).
"""
