"""Maximum-Tsallis-entropy threshold segmentation of CT volumes on MI355X.

The compute path is a hand-written HIP library (``libts.so``, C ABI declared
in ``include/ts.h``); ``paper_2012_10684_amd.api`` only marshals arguments to
it.  Importing this package loads nothing: import ``.api`` to load the
library (it fails loudly if the library has not been built) and ``.synth``
for the seeded synthetic CT generator.
"""
