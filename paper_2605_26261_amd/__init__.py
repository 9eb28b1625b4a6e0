"""MI355X-native FTLM hot path for spin-1/2 Heisenberg clusters.

``ftlm`` is the binding of the C-ABI library libftlm.so (HIP kernels for
gfx950 plus host C++); ``driver`` strings its calls into a full FTLM run.
"""
