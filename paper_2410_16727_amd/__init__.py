"""MI355X-native batched seeded trajectory optimisation (the optimiser stage
of DiffusionSeeder, arXiv 2410.16727, Sec. 4.4 / App. A.6).

``dsopt`` is the ctypes binding of the gfx950 library ``libdsopt.so``;
``autograd`` exposes the objective as a torch.autograd.Function."""
from . import dsopt  # noqa: F401
