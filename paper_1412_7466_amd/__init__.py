"""MI355X-native solver for plane-wave scattering from a layered periodic grating
with many circular inclusions (Lai, Kobayashi, Barnett).

The compute path is the C-ABI library ``libgrating.so`` (hand-written HIP for
gfx950); ``paper_1412_7466_amd.grating`` is its thin ctypes binding and
``paper_1412_7466_amd.inputs`` generates seeded synthetic workloads.
"""
