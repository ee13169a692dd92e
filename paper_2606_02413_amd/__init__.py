"""MI355X-native refractive radio ray tracing with ray-tube magnification.

Submodules are imported explicitly: ``corona`` (seeded synthetic inputs),
``rtsun`` (the binding to the HIP library's C ABI), ``autograd`` (the
torch.autograd.Function over the adjoint).  Importing the package itself loads
nothing.
"""
