"""MI355X-native hot path of TV-superiorized proton-CT reconstruction
(arXiv 1803.01112): MLP row formation, block-iterative DROP and NTVS
perturbation steps as hand-written gfx950 HIP kernels behind a C ABI
(include/tvs.h), with a thin Python binding (``tvs``) and a seeded
synthetic-input generator (``synth``)."""
