"""CPU oracle for the motion-vector backward warp — TEST INFRASTRUCTURE ONLY.

A plain, slow, float64 statement of what the warp computes, used to check the
HIP path. Only the test suite, the smoke check and the benchmark's CPU
baseline may import, call, link or run anything in this package; the product
path never does, and shares no code with it.

* ``warp_oracle``: vectorised NumPy over pixels, following the definition in
  the order the method states it.
* ``scene_stats``: the per-frame motion mean and variance and the other
  scene-state quantities that accompany a warp.
* ``quality``: per-frame MSE, PSNR and SSIM of a predicted frame against
  the ground truth.
* ``decision_paths``: the decision tree of the frames shown between rendered
  frames (Table V), chained warps W(P_i), and a fixed threshold policy.
* ``warp_ref.c`` (+ ``ref_c``): the same definition as scalar C loops in
  float64, built with gcc (no HIP); used for the cross-check and as the timed
  CPU baseline.
"""
