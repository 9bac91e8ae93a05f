"""Reader for the hand-retyped closed forms under tests/golden/."""
import ast
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

_ALLOWED = (ast.Expression, ast.BinOp, ast.UnaryOp, ast.Constant, ast.Name, ast.Load,
            ast.Add, ast.Sub, ast.Mult, ast.Div, ast.Pow, ast.USub, ast.UAdd)


def _eval(expr: str, env: dict) -> float:
    tree = ast.parse(expr.strip(), mode="eval")
    for node in ast.walk(tree):
        if not isinstance(node, _ALLOWED):
            raise ValueError(f"disallowed syntax in golden expression: {expr!r}")
    return float(eval(compile(tree, "<golden>", "eval"), {"__builtins__": {}}, dict(env)))


def read_blocks(name: str) -> dict:
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                blocks[cur] = []
                continue
            blocks[cur].append([c.strip() for c in line.split("|")])
    return blocks


def evaluate(rows, **env) -> np.ndarray:
    return np.array([[_eval(c, env) for c in r] for r in rows])
