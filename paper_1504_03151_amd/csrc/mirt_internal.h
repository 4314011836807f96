// mirt_internal.h -- host-side scene object and helpers shared by the library's
// translation units.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/mirt.h"
#include "rt_common.h"

namespace mirt {

void set_error(const std::string& msg);
struct SceneHost;
// Writes the refit order of the node section (blob section off_refit) and refit_levels.
void refit_schedule(SceneHost& h);

// Host copy of a built scene: one contiguous blob laid out exactly as it is
// uploaded, plus the offsets of each section inside it.
struct SceneHost {
    std::vector<uint8_t> blob;
    size_t off_nodes = 0, off_prims = 0, off_normals = 0, off_planes = 0, off_plane_mat = 0, off_mats = 0,
           off_lights = 0, off_refit = 0;
    std::vector<int64_t> refit_levels;   // device refit: first entry of each level of the refit order (+ end)
    int n_spheres = 0, n_tris = 0, n_planes = 0, n_lights = 0, n_materials = 0;
    int64_t n_nodes = 0;
    int depth = 0, stack_size = 0;
    int layout = 0;               // RT_LAYOUT_* of the node section
    bool area_lights = false;     // some light is an area light (sampled per pass)
    std::vector<Node> bvh2;       // the binary tree as built (depth-first), source of every layout
    float scale = 1.0f;           // max(1, max |coordinate|) of the scene
    rt_scene_info info{};
    void* dev = nullptr;
    size_t dev_bytes = 0;
    uint64_t uid = 0;             // distinguishes scenes in launch caches

    DevScene view(const uint8_t* base) const {
        DevScene s;
        s.nodes = reinterpret_cast<const Node*>(base + off_nodes);
        s.nodes4 = reinterpret_cast<const Node4*>(base + off_nodes);
        s.nodes4q = reinterpret_cast<const Node4q*>(base + off_nodes);
        s.wide = layout == RT_LAYOUT_BVH4 ? 1 : (layout == RT_LAYOUT_BVH4Q ? 2 : 0);
        s.prims = reinterpret_cast<const float4*>(base + off_prims);
        s.normals = reinterpret_cast<const float4*>(base + off_normals);
        s.planes = reinterpret_cast<const float4*>(base + off_planes);
        s.plane_mat = reinterpret_cast<const int*>(base + off_plane_mat);
        s.mats = reinterpret_cast<const DevMaterial*>(base + off_mats);
        s.lights = reinterpret_cast<const DevLight*>(base + off_lights);
        s.n_spheres = n_spheres;
        s.n_tris = n_tris;
        s.n_planes = n_planes;
        s.n_lights = n_lights;
        s.n_bvh = n_spheres + n_tris;
        s.stack_size = stack_size;
        return s;
    }
    DevScene host_view() const { return view(blob.data()); }
    DevScene dev_view() const { return view(static_cast<const uint8_t*>(dev)); }
};

}  // namespace mirt

struct rt_scene {
    mirt::SceneHost h;
};
