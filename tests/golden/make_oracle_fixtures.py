"""Write the stored oracle results that the GPU parity tests compare against.

Calls only the FP64 oracle (``oracle/``) on the seeded synthetic scenes of
``paper_1504_03151_amd.scenes`` (input generation only, none of the tracer's
arithmetic).  Nothing here comes from the HIP path.

    python tests/golden/make_oracle_fixtures.py            # all fixtures
    python tests/golden/make_oracle_fixtures.py c2_frame   # one

Fixtures:

* ``c2_frame_oracle.npz`` -- the 1920x1080 x 16 jittered samples, depth-8
  icosphere field (1,000 icospheres, 1,280,000 triangles, 50/30/20 Phong /
  mirror / glass, 8 point lights), rendered by brute force on a seeded subset
  of 1,024 pixels: 512 whose first sample's camera ray hits an object and 512
  others (the frame is ~90% background).  Per pixel and sample: the primary
  hit id, the radiance and the robustness margin; per pixel: the averaged
  radiance, the margin over all 16 samples and the per-depth query counts.
  The full frame (33M camera rays x 1.28M triangles per bounce) is out of
  reach of brute force; the subset is the scale at which the oracle can still
  vouch for the benchmarked frame.

The scene, camera and render settings are hashed into the fixture
(``scene_digest``); the test refuses a fixture whose digest differs from the
workload it renders.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

C2_FRAME = os.path.join(HERE, "c2_frame_oracle.npz")
C2_PIXELS_HIT = 512
C2_PIXELS_OTHER = 512
C2_CANDIDATE_SEED = 23


def scene_digest(w) -> str:
    """SHA-256 (16 hex digits) of every array of the scene plus the camera and render settings."""
    h = hashlib.sha256()
    sc = w.scene
    for a in (sc.spheres, sc.sphere_mat, sc.tris, sc.tri_mat, sc.planes, sc.plane_mat, sc.materials, sc.lights):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    c, p = w.camera, w.params
    h.update(repr((tuple(c.eye), tuple(c.look_at), tuple(c.up), float(c.vfov_deg), c.width, c.height)).encode())
    h.update(repr((p.spp, p.max_depth, p.jitter, int(p.seed), p.frame, tuple(p.bg), float(p.eps), p.gi)).encode())
    return h.hexdigest()[:16]


def make_c2_frame(path: str = C2_FRAME) -> None:
    import oracle
    from paper_1504_03151_amd import scenes as S

    w = S.config2()
    t0 = time.time()
    cand = S.pixel_subset(w.camera, 12000, C2_CANDIDATE_SEED)
    o, d = oracle.camera_rays(w.camera, w.params, cand, sample=0)
    _, ih, _ = oracle.closest(w.scene, o, d)
    hit, other = cand[ih >= 0], cand[ih < 0]
    assert len(hit) >= C2_PIXELS_HIT and len(other) >= C2_PIXELS_OTHER
    pixels = np.sort(np.concatenate([hit[:C2_PIXELS_HIT], other[:C2_PIXELS_OTHER]]))
    print(f"c2 subset: {len(pixels)} pixels ({time.time() - t0:.0f} s)", flush=True)
    ref = oracle.render(w.scene, w.camera, w.params, pixels)
    print(f"c2 render: {time.time() - t0:.0f} s; per-sample robust fraction "
          f"{(ref['margin_s'] > 1e-4).mean():.4f}, pixel {(ref['margin'] > 1e-4).mean():.4f}", flush=True)
    np.savez_compressed(
        path, digest=np.array(scene_digest(w)), pixels=pixels.astype(np.int64),
        ids=ref["ids"].astype(np.int32), rgb_s=ref["rgb_s"].astype(np.float32),
        margin_s=ref["margin_s"].astype(np.float32), rgb=ref["rgb"].astype(np.float32),
        margin=ref["margin"].astype(np.float32), counts=ref["counts"].astype(np.int32))
    print(f"wrote {path} ({os.path.getsize(path) / 1024:.0f} KiB)", flush=True)


FIXTURES = {"c2_frame": make_c2_frame}

if __name__ == "__main__":
    names = sys.argv[1:] or list(FIXTURES)
    for n in names:
        FIXTURES[n]()
