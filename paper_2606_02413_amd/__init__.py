"""MI355X-native refractive radio ray tracing with ray-tube magnification.

Submodules are imported explicitly: ``corona`` (seeded synthetic inputs),
``rtsun`` (the binding to the HIP library's C ABI, including the
torch.autograd.Function over the adjoint, ``rtsun.rtsun_function()``),
``fitting`` (a parameterised corona fitted to maps through that Function).
Importing the package itself loads nothing.
"""
