"""MI355X-native patch-guided nested-dissection ordering (gfx950 HIP).

``fastperm`` holds the binding of libfastperm.so (C ABI in include/fastperm.h);
``meshgen`` holds the seeded synthetic mesh patterns used as inputs.
"""
