"""MI355X-native coupled D3Q19-MRT / D3Q7-MRT thermal lattice Boltzmann step
(Xu, Shi & Xi 2019, arXiv:1903.08882).

The compute path is the HIP library built from ``csrc/`` (C ABI declared in
``include/lbm.h``); ``binding`` marshals arguments to it, with PyTorch used for
device memory and streams only.  ``synth`` holds the seeded input generators.
Importing this package loads nothing; ``binding`` loads the library.
"""
