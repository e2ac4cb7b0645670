"""MI355X (gfx950) motion-blur differentiable rasterizer with the fast
barycentric coordinate solver (arXiv 2602.07860).

Modules:
  binding   ctypes binding of the C ABI (include/motion_blur_raster.h)
  render    PyTorch front end: render_forward / render_backward / BlurRender
  workloads seeded synthetic meshes, cameras and motions
  build     hipcc build of the in-tree HIP library
"""
__all__ = ["binding", "render", "workloads", "build"]
