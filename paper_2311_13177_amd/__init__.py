"""MI355X-native lifted-PROPELLER reconstruction: HIP kernels behind a C ABI (libvp.so).

``binding`` holds the ctypes binding with the C names; ``autograd`` wraps the forward
model and its adjoint as a ``torch.autograd.Function``; ``build`` compiles the library.
"""

__all__ = ["binding", "autograd", "build"]
