"""The allocation-free refit entry point (rt_scene_refit_noalloc) against rt_scene_refit.

The no-alloc form takes its scratch (refit header and a box per node) from the
library's static device buffer instead of a caller workspace.  Two calls in a
row, the second on a smaller scene, must each give the blob the workspace form
gives, bit for bit; invalid input is reported and changes nothing; a scene
whose scratch exceeds the buffer is refused before any device work.
"""
import copy

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1504_03151_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_03151_amd import rt as _rt
    _rt.lib()
    return _rt


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _moved(scene, seed, shift=0.6, jitter=0.05):
    rng = np.random.default_rng(seed)
    s = copy.deepcopy(scene)
    if len(s.spheres):
        s.spheres = s.spheres.copy()
        s.spheres[:, :3] += rng.uniform(-shift, shift, (len(s.spheres), 3)).astype(np.float32)
        s.spheres[:, 3] *= rng.uniform(0.8, 1.2, len(s.spheres)).astype(np.float32)
    if len(s.tris):
        s.tris = (s.tris + rng.uniform(-shift, shift, (len(s.tris), 1, 3))
                  + rng.normal(0.0, jitter, s.tris.shape)).astype(np.float32)
    return s


def test_noalloc_refit_equals_workspace_refit(rt):
    big = S.config2(n_objects=300).scene                              # 384,000 triangles
    small = S.random_tiny(3, n_spheres=9, n_tris=300, size=8).scene   # spheres and triangles
    for scene, layout, seed in ((big, rt.LAYOUT_BVH4Q, 1), (small, rt.LAYOUT_DFS, 2)):
        print(f"noalloc refit: {len(scene.tris)} triangles, {len(scene.spheres)} spheres, layout {layout}", flush=True)
        a = rt.Scene(scene, node_layout=layout).upload()
        b = rt.Scene(scene, node_layout=layout).upload()
        before = b.device_blob().clone()
        m = _moved(scene, seed)
        sp = _dev(m.spheres) if len(m.spheres) else None
        tr = _dev(m.tris) if len(m.tris) else None
        a.refit(sp, tr, sync=True)
        b.refit(sp, tr, sync=True, noalloc=True)
        torch.cuda.synchronize()
        assert not torch.equal(b.device_blob(), before)               # the geometry moved
        assert torch.equal(a.device_blob(), b.device_blob())
    # invalid positions: reported with FLAG_SYNC, the blob unchanged; the next valid call works again
    snap = b.device_blob().clone()
    bad = _moved(small, 3)
    bad.tris[5, 1, 2] = np.nan
    with pytest.raises(rt.RTError, match="INVALID_ARG"):
        b.refit(_dev(bad.spheres), _dev(bad.tris), sync=True, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(b.device_blob(), snap)
    b.refit(_dev(small.spheres), _dev(small.tris), sync=True, noalloc=True)
    ref = rt.Scene(small, node_layout=rt.LAYOUT_DFS).upload()
    torch.cuda.synchronize()
    assert torch.equal(b.device_blob(), ref.device_blob())           # identity refit: the upload, bit for bit


def test_noalloc_refit_refuses_scenes_beyond_its_buffer(rt):
    cap = rt.lib().rt_scene_refit_noalloc_max_bytes()
    assert cap == 32 << 20
    w = S.config2(n_objects=1100)                                     # 1,408,000 triangles, one per leaf
    sc = rt.Scene(w.scene, leaf_max=1)
    need = rt.lib().rt_scene_refit_workspace_bytes(sc.handle)
    assert need > cap, (need, cap)
    rc = rt.lib().rt_scene_refit_noalloc(sc.handle, None, None, 0, None)
    assert rc == -5 and b"more than the" in rt.lib().rt_last_error()
