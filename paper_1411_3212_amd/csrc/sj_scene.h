// Scene internals used by the serving runtime (same library).
#pragma once

#include "sj.h"
#include "sj_device.h"

// Enqueues a copy of the scene's control block to pinned host memory.
int sj_scene_ctl_to_host_async(sj_scene *scene, sj::Ctl *h_ctl);
// Adopts a control block copied after the scene's last tick (its stream has
// passed the copy): the next tick's quadtree decision is then made on the host.
void sj_scene_ctl_from_host(sj_scene *scene, const sj::Ctl *h_ctl);
// Status of the last tick from the adopted control block.
int sj_scene_status(sj_scene *scene);
// Enqueues a copy of the scene's positions by id (capacity_objects float2,
// NaN: no position yet) to (to_host != 0) or from pinned host memory.
int sj_scene_positions_copy(sj_scene *scene, void *h_pos, int to_host);
// Message returned by sj_last_error(NULL) (creation and the calls that take
// no scene).
void sj_set_global_error(const char *fmt, ...);
