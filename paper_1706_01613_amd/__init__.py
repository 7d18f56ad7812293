"""hexval: MI355X-native validity test of linear hexahedra.

The library is ``libhexval.so`` (hand-written HIP for gfx950) behind a C ABI
(``include/hexval.h``); ``paper_1706_01613_amd.hexval`` is its thin Python
binding.  ``paper_1706_01613_amd.synth`` holds the seeded input generators.
Importing the package loads nothing; the binding loads the library on first use
and raises if it has not been built.
"""
