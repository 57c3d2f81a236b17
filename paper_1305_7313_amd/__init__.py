"""MI355X-native exact-exchange (Fock) band-pair path.

The compute lives in ``libfockx.so`` (hand-written HIP kernels for gfx950
behind the C ABI declared in ``include/fock.h``).  ``fock`` is the thin
ctypes binding with the same names; ``autograd`` wraps the exchange energy
in a ``torch.autograd.Function``; ``batch`` is the batched form.
"""
