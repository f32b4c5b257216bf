"""paper_1308_1464_amd: MI355X-native 2D wave-propagation step (HIP, gfx950).

The compute path is the C-ABI library ``libmanyclaw.so`` (hand-written HIP
kernels); ``manyclaw`` is its thin ctypes binding.  The library is loaded on
first use and a missing or unloadable library raises an error: there is no
CPU fallback.
"""
