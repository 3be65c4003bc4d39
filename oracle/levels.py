"""Index and overlap maps of one level (section 2.1; recursion of section 2.2).

Readings of the paper used here (the paper does not fix them):
  * overlap = delta layers of the node graph of the level (delta = 1 means one
    layer of nodes beyond the closure of the part's elements);
  * a local block holds the free velocity dofs of the overlapping node set and
    the pressure dofs of the part's own elements;
  * the interface is the set of nodes with a free dof that belong to elements of
    at least two parts; an interface entity is a maximal connected (in the node
    graph) set of interface nodes with the same set of parts;
  * with discontinuous pressure, the constant pressure mode of each element is an
    interface dof (one pressure coarse column per part, its constants), the
    linear modes are interior dofs;
  * coarse dofs are numbered entity-major / direction-minor, then one pressure
    column per part;
  * the mesh of the next level has the entities as nodes (3 dofs each) and the
    parts as elements (one constant pressure each); two entities are adjacent if
    some of their nodes are.
"""
from collections import deque

import numpy as np

VERTEX, EDGE, FACE = 0, 1, 2


class Mesh:
    """One level: nodes with up to 3 velocity dofs, elements with nodes and 4 pressure slots."""

    def __init__(self, n_dof, node_dof, elem_nodes, elem_pdof, elem_part, n_parts, adj):
        self.n_dof = int(n_dof)
        self.node_dof = np.asarray(node_dof, dtype=np.int64).reshape(-1, 3)
        self.n_nodes = self.node_dof.shape[0]
        self.elem_nodes = [tuple(int(v) for v in en) for en in elem_nodes]
        self.elem_pdof = np.asarray(elem_pdof, dtype=np.int64).reshape(-1, 4)
        self.elem_part = np.asarray(elem_part, dtype=np.int64)
        self.n_parts = int(n_parts)
        self.adj = adj                      # list of sets of node ids


def level1_mesh(problem):
    """Level-1 mesh: node graph links nodes of one element whose lattice offsets differ by <= 1 per axis."""
    ne = problem.n_elem
    en = problem.elem_node.reshape(ne, 27)
    k = np.arange(27)
    off = np.stack([k % 3, (k // 3) % 3, k // 9], axis=1)
    pairs = [(a, b) for a in range(27) for b in range(27)
             if a != b and np.all(np.abs(off[a] - off[b]) <= 1)]
    adj = [set() for _ in range(problem.n_nodes)]
    for e in range(ne):
        nodes = en[e]
        for a, b in pairs:
            adj[nodes[a]].add(int(nodes[b]))
    return Mesh(problem.n, problem.node_dof, en, problem.elem_pdof, problem.elem_part,
                problem.n_parts[0], adj)


class LevelMaps:
    pass


def build_level(mesh, delta=1, pressure_gamma="constants"):
    """All index maps of one level, straight from the definitions.

    pressure_gamma="constants": the constant pressure mode of every element is an
    interface dof, the linear modes are interior dofs of their part (saddle-point
    extension); "all": every pressure mode is an interface dof (the linear modes
    belong to no coarse column), so the extension into the interior is
    velocity-only.  The coarse columns are the same either way."""
    m = LevelMaps()
    N = mesh.n_parts
    part_elems = [[] for _ in range(N)]
    for e, p in enumerate(mesh.elem_part):
        part_elems[p].append(e)
    # S(v): parts of the elements that contain v
    S = [set() for _ in range(mesh.n_nodes)]
    for e, nodes in enumerate(mesh.elem_nodes):
        for v in nodes:
            S[v].add(int(mesh.elem_part[e]))
    has_free = (mesh.node_dof >= 0).any(axis=1)
    gamma = [v for v in range(mesh.n_nodes) if has_free[v] and len(S[v]) >= 2]
    m.S = S
    m.gamma_nodes = np.array(gamma, dtype=np.int64)
    # entities: equal-S classes split into connected components
    classes = {}
    for v in gamma:
        classes.setdefault(frozenset(S[v]), set()).add(v)
    ents = []
    for key, members in classes.items():
        left = set(members)
        while left:
            start = min(left)
            comp = {start}
            queue = deque([start])
            left.discard(start)
            while queue:
                u = queue.popleft()
                for w in mesh.adj[u]:
                    if w in left:
                        left.discard(w)
                        comp.add(w)
                        queue.append(w)
            ents.append((min(comp), sorted(comp), key))
    ents.sort(key=lambda t: t[0])
    m.entities = [np.array(c, dtype=np.int64) for _, c, _ in ents]
    m.entity_parts = [sorted(k) for _, _, k in ents]
    kinds = []
    for (_, c, k) in ents:
        if len(c) == 1:
            kinds.append(VERTEX)
        elif len(k) == 2:
            kinds.append(FACE)
        else:
            kinds.append(EDGE)
    m.entity_kind = np.array(kinds, dtype=np.int64)
    # coarse columns: (entity, direction) with at least one free dof, then one pressure column per part
    col_entity, col_dir, col_dofs = [], [], []
    ent_col = -np.ones((len(ents), 3), dtype=np.int64)
    for E, nodes in enumerate(m.entities):
        for d in range(3):
            dofs = [int(mesh.node_dof[v, d]) for v in nodes if mesh.node_dof[v, d] >= 0]
            if dofs:
                ent_col[E, d] = len(col_dofs)
                col_entity.append(E)
                col_dir.append(d)
                col_dofs.append(sorted(dofs))
    part_col = -np.ones(N, dtype=np.int64)
    for i in range(N):
        dofs = sorted(int(mesh.elem_pdof[e, 0]) for e in part_elems[i] if mesh.elem_pdof[e, 0] >= 0)
        if dofs:
            part_col[i] = len(col_dofs)
            col_entity.append(-1 - i)
            col_dir.append(3)
            col_dofs.append(dofs)
    m.col_entity = np.array(col_entity, dtype=np.int64)
    m.col_dir = np.array(col_dir, dtype=np.int64)
    m.col_dofs = col_dofs
    m.ent_col = ent_col
    m.part_col = part_col
    m.n_coarse = len(col_dofs)
    # overlapping dof sets D_i and interior sets I_i
    dom, inter = [], []
    for i in range(N):
        closure = set()
        for e in part_elems[i]:
            closure.update(mesh.elem_nodes[e])
        layer = set(closure)
        frontier = set(closure)
        for _ in range(delta):
            new = set()
            for u in frontier:
                new.update(w for w in mesh.adj[u] if w not in layer)
            layer |= new
            frontier = new
        dofs = set()
        for v in layer:
            dofs.update(int(x) for x in mesh.node_dof[v] if x >= 0)
        for e in part_elems[i]:
            dofs.update(int(x) for x in mesh.elem_pdof[e] if x >= 0)
        dom.append(np.array(sorted(dofs), dtype=np.int64))
        idofs = set()
        for v in closure:
            if S[v] == {i}:
                idofs.update(int(x) for x in mesh.node_dof[v] if x >= 0)
        if pressure_gamma == "constants":
            for e in part_elems[i]:
                idofs.update(int(x) for x in mesh.elem_pdof[e, 1:] if x >= 0)
        inter.append(np.array(sorted(idofs), dtype=np.int64))
    m.dom = dom
    m.inter = inter
    m.part_elems = part_elems
    gdofs = set()
    for v in gamma:
        gdofs.update(int(x) for x in mesh.node_dof[v] if x >= 0)
    for e in range(len(mesh.elem_nodes)):
        modes = mesh.elem_pdof[e] if pressure_gamma == "all" else mesh.elem_pdof[e, :1]
        gdofs.update(int(x) for x in modes if x >= 0)
    m.gamma_dofs = np.array(sorted(gdofs), dtype=np.int64)
    return m


def next_mesh(mesh, maps, part_parent, n_parts_next):
    """Mesh of the next level: entities become nodes, parts become elements."""
    n_ent = len(maps.entities)
    elem_nodes = [[] for _ in range(mesh.n_parts)]
    for E, parts in enumerate(maps.entity_parts):
        for i in parts:
            elem_nodes[i].append(E)
    ent_of = {}
    for E, nodes in enumerate(maps.entities):
        for v in nodes:
            ent_of[int(v)] = E
    adj = [set() for _ in range(n_ent)]
    for u, E in ent_of.items():
        for w in mesh.adj[u]:
            F = ent_of.get(w)
            if F is not None and F != E:
                adj[E].add(F)
    elem_pdof = -np.ones((mesh.n_parts, 4), dtype=np.int64)
    elem_pdof[:, 0] = maps.part_col
    return Mesh(maps.n_coarse, maps.ent_col, [sorted(x) for x in elem_nodes], elem_pdof,
                part_parent, n_parts_next, adj)
