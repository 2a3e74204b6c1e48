"""MI355X-native hybrid compressor for velocity-space histograms.

`paper_2212_10733_amd.hcz` binds the HIP library (libhcz.so, C ABI in include/hcz.h);
`paper_2212_10733_amd.synth` draws the seeded synthetic inputs.  Importing the package
loads neither.
"""
