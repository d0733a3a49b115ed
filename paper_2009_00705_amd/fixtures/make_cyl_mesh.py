"""Write cyl_mesh.npz: the seeded Delaunay cylinder mesh of the unstructured
workloads (12,015 triangles in [-4, 4]^2 around a cylinder of radius 0.5),
frozen so that its numbering does not depend on the Delaunay implementation
of the machine that runs the workloads.

    python -m paper_2009_00705_amd.fixtures.make_cyl_mesh
"""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "cyl_mesh.npz")


def main() -> None:
    from paper_2009_00705_amd.workloads import cylinder_mesh
    m = cylinder_mesh()
    np.savez_compressed(PATH, xy=m["xy"], tri=m["tri"], edge_tag=m["edge_tag"], curved_edge=m["curved_edge"],
                        circle=m["circle"], n_layers=np.int32(m["n_layers"]), depth=np.float64(m["depth"]))
    print(f"wrote {PATH}: {m['tri'].shape[0]} triangles, {m['xy'].shape[0]} vertices")


if __name__ == "__main__":
    main()
