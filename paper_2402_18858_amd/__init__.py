"""MI355X (gfx950) chemistry advance: DI and ANN paths behind a C ABI.

``chemk`` is the binding of libchemk.so (include/chemk.h); ``train`` drives
training-data generation and network training through the same library."""
