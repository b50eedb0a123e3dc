"""CPU oracle for the S3R-GS per-view rendering step (arXiv 2503.08217).

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import or run anything in this package.
The GPU product path never calls it, and it shares no code with the HIP
library: no kernels, headers, helpers, constants or pre/post-processing.  The
only thing both sides consume is the seeded input generator in `scenes/`,
which holds none of the method's arithmetic.

What it computes, and how it is organised
-----------------------------------------
* `frames`    time normalisation (Sec. 3.3 "Temporal separation"), instance
              cameras W_{t,i} = W_t W_{t,i2g} (Sec. 3.3 "Instance-specific
              projection"), and the conventional local->global transform
              (Sec. 3.1).  FP64.
* `project64` the conventional route in FP64: transform every instance
              Gaussian to the world frame, then project with W_t, K_t (Eq. 1).
              This is the value layer and the reference for gradients.
* `decide32`  the streamlined route in IEEE binary32 with one fixed operation
              order (each + - * / sqrt rounded, no fused multiply-add).  It
              produces every discrete decision (temporal pass, visible mask M_t,
              LOD cull, footprint rectangle, depth key) in the precision the
              GPU kernels decide in, so the two can be compared bit for bit.
* `sh`        the real spherical-harmonic colour model (Sec. 3.1), built from
              scipy's complex spherical harmonics and, separately, from the
              explicit normalised polynomials.
* `order`     depth/tile order of contributors.
* `composite` per-pixel front-to-back alpha blending (Eq. 2) in FP64, with a
              scalar brute-force twin for tiny inputs.
* `visibility` point-life update, fold and reset (Eqs. 5-6).
* `grad`      reference gradients by torch-CPU FP64 autograd with every
              discrete decision frozen.
* `render`    top-level per-view driver tying the layers together.

Parity status of each function is stated in its docstring; readings of the
paper where it is silent or garbled are listed in `READINGS` below.
"""

READINGS = {
    "time": "rendering time normalised to [-1,1] as t = -1 + 2*tau/(T-1)",
    "static_id": "instance id 0 marks static Gaussians (pose = identity)",
    "covariance": "Sigma in R^3 (garbled) read as 3DGS scale s and quaternion q (w,x,y,z)",
    "jacobian": "J of Eq. (1) read as the EWA affine approximation of the perspective map",
    "perspective": "mu' = K_t W_t mu read with the perspective divide",
    "mask": "M_t = frustum-visible mask taken before the LOD cull",
    "lod_scale": "2D scale = sqrt of the largest eigenvalue of the undilated 2D covariance",
    "lod_drop": "drop probability p = 1 for sub-threshold Gaussians (Eq. 7 with p_max = 1, D -> 0+)",
    "order": "contributors ordered by (depth bits, Gaussian id) ascending",
    "cutoff": "pixels with Mahalanobis power below -4.5 skip the Gaussian",
    "fold": "point life kept across FOLD; RESET restores v=(-1,1), l=(1,-1)",
    "colour": "real SH of degree <= 3, 3DGS sign convention, +0.5 offset, clamp at 0",
}
