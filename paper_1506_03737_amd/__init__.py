"""MI355X-native particle-mesh COLA time step (L-PICOLA, Howlett, Manera & Percival 2015).

The method lives in liblpc.so (hand-written HIP for gfx950 behind the C ABI of include/lpc.h); `lpc` is its thin
Python binding. Build with `python -m paper_1506_03737_amd.build`.
"""
