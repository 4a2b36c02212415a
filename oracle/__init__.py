"""Plain, slow FP64 CPU oracle of the crowd-splatting hot path.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. The GPU library never
calls it, never links it and never falls back to it.

Every function works in float64 on the generator's float32 arrays (upcast)
and follows the method step by step in the order the paper and the work it
builds on state them:

* ``skinning``  forward kinematics and linear blend skinning of the shared
                template means and covariances (CrowdSplat §2, Fig. 2, stage 2);
* ``splat``     EWA projection, SH colour, opacity-aware footprint, tile
                binning keys, the stable (tile|depth) sort and front-to-back
                compositing (3D Gaussian Splatting, Kerbl et al. 2023, which
                CrowdSplat §2 uses as its renderer);
* ``lod``       fixed-distance level of detail (CrowdSplat §2, last paragraph)
                and the learned-LoD network (features, MLP, Adam, PSNR labels);
* ``grad``      the analytic backward of the renderer and the fit loss.

It shares no code, constants or helpers with the GPU library.
"""
