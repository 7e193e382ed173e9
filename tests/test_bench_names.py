"""bench.py has no name that is read but never bound.

A static walk with ``ast`` (no GPU, nothing run): every name a function reads
must be bound in that function, in an enclosing function, at module level or
among the builtins.  Comprehension and lambda targets count as bound in the
function that holds them, which can only hide a mistake, never invent one.
"""
import ast
import builtins
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["bench.py", "__graft_entry__.py"]


def _bound_in(body_nodes, args=None):
    """Names bound directly in a scope (not inside nested function bodies)."""
    names = set()
    if args is not None:
        for a in args.posonlyargs + args.args + args.kwonlyargs:
            names.add(a.arg)
        if args.vararg:
            names.add(args.vararg.arg)
        if args.kwarg:
            names.add(args.kwarg.arg)
    stack = list(body_nodes)
    while stack:
        n = stack.pop()
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            names.add(n.name)
            stack.extend(n.decorator_list)
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
            names.add(n.id)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            for a in n.names:
                names.add((a.asname or a.name).split(".")[0])
        elif isinstance(n, ast.ExceptHandler) and n.name:
            names.add(n.name)
        elif isinstance(n, (ast.Global, ast.Nonlocal)):
            names.update(n.names)
        elif isinstance(n, ast.Lambda):
            a = n.args
            for x in a.posonlyargs + a.args + a.kwonlyargs:
                names.add(x.arg)
        stack.extend(ast.iter_child_nodes(n))
    return names


def _loads(body_nodes):
    """(name, line) read directly in a scope (not inside nested function bodies)."""
    out = []
    stack = list(body_nodes)
    while stack:
        n = stack.pop()
        if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            stack.extend(n.decorator_list)
            if not isinstance(n, ast.ClassDef):
                stack.extend(d for d in n.args.defaults + n.args.kw_defaults if d is not None)
            continue
        if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load):
            out.append((n.id, n.lineno))
        stack.extend(ast.iter_child_nodes(n))
    return out


def undefined_names(src: str):
    tree = ast.parse(src)
    known = set(dir(builtins)) | {"__file__", "__name__"}
    bad = []

    def visit(body, args, outer):
        scope = outer | _bound_in(body, args)
        for name, line in _loads(body):
            if name not in scope:
                bad.append((name, line))
        stack = list(body)
        while stack:
            n = stack.pop()
            if isinstance(n, (ast.FunctionDef, ast.AsyncFunctionDef)):
                visit(n.body, n.args, scope)
                continue
            if isinstance(n, ast.ClassDef):
                visit(n.body, None, scope)
                continue
            stack.extend(ast.iter_child_nodes(n))

    visit(tree.body, None, known)
    return sorted(set(bad), key=lambda x: x[1])


@pytest.mark.parametrize("name", FILES)
def test_no_unbound_names(name):
    with open(os.path.join(ROOT, name)) as f:
        bad = undefined_names(f.read())
    assert not bad, f"{name}: names read but never bound: {bad}"


def test_checker_finds_a_planted_name():
    src = "def f(a):\n    x = a + 1\n    return x + missing\n\ndef g():\n    def h():\n        return y\n    y = 2\n    return h\n"
    assert undefined_names(src) == [("missing", 3)]
