"""MI355X (gfx950) implementation of single-projection volumetric
reconstruction and tumour localisation under a PCA lung-motion model
(Li et al., "Real-time volumetric image reconstruction and 3D tumor
localization based on a single x-ray projection image for lung cancer
radiotherapy").

The computation lives in the HIP library libpcr.so (C ABI: include/pcr.h);
`paper_1004_0014_amd._lib` is its ctypes binding.  `synth` builds seeded
synthetic inputs.  Importing the package loads nothing.
"""
__version__ = "0.1.0"
