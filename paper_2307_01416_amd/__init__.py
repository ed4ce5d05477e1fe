"""MI355X-native virtual-particle Monte Carlo transport of proton pencil beams
through a range shifter and a brass aperture block (arXiv 2307.01416).

``vpmc`` is the ctypes binding of the HIP library ``libvpmc.so`` (C ABI in
``include/vpmc.h``); ``inputs`` builds seeded synthetic workloads.
"""
__all__ = ["inputs", "vpmc"]
